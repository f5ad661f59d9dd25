// fit.hip -- device L-BFGS driver of pd_fit (Section 5.2).
//
// Maximises Phi (minimises f = -Phi) for a batch of maps.  All vectors, the
// L-BFGS memory and the line-search state live on the device; one "step" is a
// fixed sequence of kernels -- objective+gradient at the trial point (with the
// pending accuracy check of the accepted iterate in the same launch), then the
// decision, which also forms the next trial point -- captured once as a HIP
// graph and replayed.  The host only polls a per-map activity flag every few
// replays.
//
// Algorithm (the paper names L-BFGS [Liu-Nocedal 1989] and nothing more; these
// are the library's documented choices): memory m, H0 = gamma I with
// gamma = s.y / y.y of the newest stored pair, first trial step 1/||g||_2 when the
// memory is empty and 1 otherwise, strong-Wolfe line search with bracketing by
// doubling and zoom by safeguarded cubic interpolation (Nocedal-Wright
// Algorithms 3.5/3.6, c1 = 1e-4, c2 = 0.9, <= 20 evaluations), pairs stored only
// if s.y > 1e-10 ||s|| ||y||, a failed search clears the memory and retries once.
// If a search exhausts its evaluations at a point with sufficient decrease, that
// point is accepted (it is evaluated once more, which the evaluation count shows).
// Gauge (Remark 4.3): LAST_ZERO zeroes grain N-1's gradient row (theta_{N-1}
// stays 0; a given start is first shifted by -theta_{N-1}, Lemma 4.2); CENTERED
// subtracts the grain mean.
#include "pd_host.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <cmath>
#include <vector>

#define FIT_THREADS 512
#define LS_C1 1e-4
#define LS_C2 0.9
#define LS_MAX_EVALS 20
#define CURV_EPS 1e-10
#define FIT_MAX_HISTORY 32
#define FIT_GRAPH_STEPS 8
// maps with at least this many unknowns run the n-length passes of an accepted
// step on several blocks (FIT_SPLIT_CHUNK elements each)
#define FIT_SPLIT_MIN_NK 1024
#define FIT_SPLIT_CHUNK 512
#define FIT_PART_W (5 * FIT_MAX_HISTORY + 8)
// elements per thread whose loads a one-block vector pass issues together
#define FIT_UNROLL 4
// format tag of a saved L-BFGS state (first header entry)
#define FIT_STATE_TAG 20605.0

enum { PH_INIT = 0, PH_BRACKET = 1, PH_ZOOM = 2, PH_ACCEPT_NEXT = 3, PH_STOP = 4 };
enum { ST_RUNNING = -1, ST_TARGET = 0, ST_BUDGET = 1, ST_GTOL = 2, ST_LSFAIL = 3, ST_NONFINITE = 4 };

struct FitDev {
  int32_t N, K, NK, m, max_iter, check_every, gauge;
  int32_t vt;  // threads that own elements (from this map's size alone); others add zeros
  int64_t n_pix;
  double target_acc, gtol;
  double *x, *g, *d, *xt, *graw, *S, *Y, *rho;
  double *SY, *YY, *Sg, *Yg;  // Gram matrices s_j.y_k, y_j.y_k over the m+1 ring slots; S^T g, Y^T g
  const double *phi_t;
  const int64_t *part_c;  // per-block correct counts of the last assignment
  int32_t c_items;        // their number
  // certified accuracy (FP64/FP32 evaluations): the objective launch at xt also
  // counts the pixels that F_xt labels correctly (per-wave counts in part_c plus
  // the canonical pass's fb_count), so the accuracy of an accepted iterate is
  // known when it is accepted; the decision kernel clears the slots for the next
  // evaluation.  Otherwise (BF16) the accepted iterate is assigned in the next
  // step (assign_pending).
  int32_t cert;
  int64_t cnt_t;          // correct pixels of the evaluation at xt
  double *cert_slot;
  int32_t *unc_count;
  int64_t *fb_count;
  double *thc;       // evaluation input: cscale * (xt - grain mean of xt)
  double cscale;     // -log2(e) / eps
  int32_t *active, *assign_pending;
  // diagonal preconditioner (precond = refresh period T, 0 = off): Dinv =
  // 1 / (diag + floor max diag) from the evaluation's Hessian diagonal
  int32_t precond;
  int32_t *want_diag;   // read by the gradient kernels: compute diag this evaluation
  const double *diag;
  double *Dinv;
  double diag_floor;
  // state
  int32_t status, phase, iters, evals, ls_evals, hist_len, hist_head, reset_tried;
  double f, t, f0, dphi0, gamma, acc, gg, gmax;
  double prev_t, prev_f, prev_d, lo_t, lo_f, lo_d, hi_t, hi_f, hi_d;
  uint64_t clk_start, clk_target;
  // device clock at the decision on the first evaluation and at the last accepted
  // iterate, and the evaluation count at that iterate (the report's step timing)
  uint64_t clk_first, clk_last;
  int32_t evals_last;
  uint64_t *trace;  // optional stage stamps of the decision kernel (PD_FIT_TRACE builds)
  // per-iteration metrics ring of the caller (pd_fit_opts.trace; NULL = off):
  // iterate k = rec_base + iters goes to row (k - 1) % rec_cap
  double *rec;
  int32_t rec_cap, rec_base, rec_evals;  // rec_evals: evaluations of earlier levels
  // the memory, gamma, D^-1 and the iteration count were loaded from a saved
  // state: the start keeps them and takes its direction from the stored pairs
  int32_t resumed;
  // multi-block passes of an accepted step (maps with N K >= FIT_SPLIT_MIN_NK):
  // phase 1 = the memory's dot products are pending (k_fit_dots, k_fit_rec),
  // phase 2 = the direction is pending (k_fit_dir, k_fit_start)
  int32_t split, split_phase, sp_put, sp_stored, sp_refresh, nchunk;
  double sp_sy;
  double *coef_g;  // [8 * (FIT_MAX_HISTORY + 1)] recursion coefficients
  double *part;    // [nchunk][FIT_PART_W] per-block partial sums
};

#ifdef PD_FIT_TRACE
#define FIT_STAMP(F, k)                                                          \
  do {                                                                           \
    if ((F).trace && threadIdx.x == 0) (F).trace[((F).evals & 255) * 16 + (k)] = clock64(); \
  } while (0)
#else
#define FIT_STAMP(F, k) do { } while (0)
#endif

// Doubles of a saved state after its header up to D^-1: the ring of s and y
// (m + 1 slots of N K each), rho (m + 1) and the two Gram matrices ((m + 1)^2
// each), laid out as in the fit's own vectors.
static inline size_t fit_state_ring(size_t NK, int m) {
  const size_t M1 = (size_t)m + 1;
  return 2 * M1 * NK + M1 + 2 * M1 * M1;
}

extern "C" int64_t pd_fit_state_size(int32_t n_grains, int32_t degree, int32_t history) {
  if (n_grains < 2 || degree < 1 || degree > PD_MAX_DEGREE || history < 1 || history > FIT_MAX_HISTORY)
    return 0;
  const size_t NK = (size_t)n_grains * ((degree + 1) * (degree + 2) / 2);
  return (int64_t)(PD_FIT_STATE_HEADER + fit_state_ring(NK, history) + NK);
}

struct FitState {
  hipStream_t stream = nullptr;
  double *phi_buf = nullptr;  // Phi at the maps' own eps after an annealed fit
  size_t phi_cap = 0;
};

// ------------------------------------------------------------------ block helpers
//
// Vector work is spread over the block (thread t owns elements t, t + blockDim,
// ...).  Sums use DPP wave sums and then the wave partials in wave order, so
// every reduction has a fixed order.  Up to VG dot products are accumulated in
// one pass over memory.

#define VG 16
#define MAX_WAVES (FIT_THREADS / PD_WAVE)

// Per-wave transposition space of the many-value block sums: 8 values x 64
// lanes per wave.
__shared__ double fit_xs[MAX_WAVES * 8 * PD_WAVE];

// Per-element vectors of a single-block map (N K < FIT_SPLIT_MIN_NK) during an
// accepted step, kept in LDS: the new gradient, s, y and the metric weights
// Dinv (or 1) (read by every wave's dot products), the new iterate and
// direction (read when the next trial point is formed) and that trial point
// (read for its grain means).
enum { FV_G = 0, FV_S, FV_Y, FV_W, FV_X, FV_D, FV_XT, FV_ROWS };
__shared__ double fit_vec[FV_ROWS][FIT_SPLIT_MIN_NK];
// nonzero while fit_vec's x and d rows hold the iterate and the search direction
__shared__ int fit_staged;

template <int G>
__device__ __attribute__((always_inline)) inline void blk_sums(double (&v)[G], double *red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  if constexpr (G < 8) {
#pragma unroll
    for (int q = 0; q < G; ++q) v[q] = pd_wave_sum(v[q]);
    if (nw == 1) return;
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < G; ++q) red[w * G + q] = v[q];
  } else {
    // 8 values at a time: the wave's 64 x 8 values go to LDS; lane l adds the
    // 8 entries (l & 7) * 8 .. +7 of value l >> 3, and a butterfly over the 8
    // lanes of its group completes the wave sum (about 35 instructions per 8
    // values instead of 160 for eight DPP wave sums).
    double *xs = fit_xs + w * 8 * PD_WAVE;
    const int q8 = lane >> 3, part = lane & 7;
    __syncthreads();  // earlier readers of red are done
#pragma unroll
    for (int c = 0; c < G; c += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) xs[u * PD_WAVE + lane] = c + u < G ? v[c + u] : 0.0;
      __syncthreads();
      const double *src = xs + q8 * PD_WAVE + part * 8;
      double t = src[0];
#pragma unroll
      for (int e = 1; e < 8; ++e) t += src[e];
      t += __shfl_xor(t, 1, PD_WAVE);
      t += __shfl_xor(t, 2, PD_WAVE);
      t += __shfl_xor(t, 4, PD_WAVE);
      if (part == 0 && c + q8 < G) red[w * G + c + q8] = t;
      __syncthreads();
    }
  }
  __syncthreads();
  // value q is summed over the waves (in wave order) by thread q, then shared
  if ((int)threadIdx.x < G) {
    double t = 0.0;
    for (int ww = 0; ww < nw; ++ww) t += red[ww * G + threadIdx.x];
    red[MAX_WAVES * 48 + threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < G; ++q) v[q] = red[MAX_WAVES * 48 + q];
}

// Maximum over the wave of a non-negative value (DPP steps as in pd_wave_sum;
// lanes outside a step's reach contribute 0).
__device__ inline double wave_max_nonneg(double v) {
  v = fmax(v, pd_dpp_f64<0x111, 0xf>(v));
  v = fmax(v, pd_dpp_f64<0x112, 0xf>(v));
  v = fmax(v, pd_dpp_f64<0x114, 0xf>(v));
  v = fmax(v, pd_dpp_f64<0x118, 0xf>(v));
  v = fmax(v, pd_dpp_f64<0x142, 0xa>(v));
  v = fmax(v, pd_dpp_f64<0x143, 0xc>(v));
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Block maximum of a non-negative value.
__device__ __attribute__((always_inline)) inline double blk_max(double v, double *red) {
  v = wave_max_nonneg(v);
  const int nw = blockDim.x >> 6;
  if (nw == 1) return v;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t = fmax(t, red[w]);
  return t;
}

// Two block sums and the block maximum of a non-negative value, in one exchange.
__device__ __attribute__((always_inline)) inline void blk_sums2_max(double (&v)[2], double &mx,
                                                                    double *red) {
  v[0] = pd_wave_sum(v[0]);
  v[1] = pd_wave_sum(v[1]);
  mx = wave_max_nonneg(mx);
  const int nw = blockDim.x >> 6;
  if (nw == 1) return;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    red[3 * w] = v[0];
    red[3 * w + 1] = v[1];
    red[3 * w + 2] = mx;
  }
  __syncthreads();
  double a = 0.0, b = 0.0, m = 0.0;
  for (int w = 0; w < nw; ++w) {
    a += red[3 * w];
    b += red[3 * w + 1];
    m = fmax(m, red[3 * w + 2]);
  }
  v[0] = a;
  v[1] = b;
  mx = m;
}

// v <- projection of v onto the gauge-fixed subspace (in place).
__device__ __attribute__((always_inline)) inline void blk_gauge(FitDev &F, double *v, double *red) {
  if (F.gauge == 0) {
    for (int k = threadIdx.x; k < F.K; k += blockDim.x) v[(size_t)(F.N - 1) * F.K + k] = 0.0;
  } else if (F.gauge == 1) {
    for (int k0 = 0; k0 < F.K; k0 += VG) {
      double sm[VG];
#pragma unroll
      for (int q = 0; q < VG; ++q) sm[q] = 0.0;
      const int cnt = min(VG, F.K - k0);
      for (int i = (int)threadIdx.x; i < F.N && (int)threadIdx.x < F.vt; i += F.vt)
#pragma unroll
        for (int q = 0; q < VG; ++q)
          if (q < cnt) sm[q] += v[(size_t)i * F.K + k0 + q];
      blk_sums<VG>(sm, red);
      for (int i = (int)threadIdx.x; i < F.N && (int)threadIdx.x < F.vt; i += F.vt)
#pragma unroll
        for (int q = 0; q < VG; ++q)
          if (q < cnt) v[(size_t)i * F.K + k0 + q] -= sm[q] / (double)F.N;
    }
  }
  __syncthreads();
}

__device__ inline double cubic_min(double a, double fa, double da, double b, double fb, double db) {
  const double lo = fmin(a, b), hi = fmax(a, b), width = hi - lo, mid = 0.5 * (a + b);
  const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - da * db;
  if (!(disc >= 0.0)) return mid;
  const double d2 = copysign(sqrt(disc), b - a);
  const double den = db - da + 2.0 * d2;
  if (den == 0.0) return mid;
  const double t = b - (b - a) * ((db + d2 - d1) / den);
  if (!(lo + 0.1 * width <= t && t <= hi - 0.1 * width)) return mid;
  return t;
}

__device__ inline void fit_stop(FitDev &F, int status) {
  F.status = status;
  *F.active = 0;
  if (F.want_diag) *F.want_diag = 0;
}

// ||g||^2, ||g||_inf and g.d of the current iterate (one pass).
__device__ __attribute__((always_inline)) inline void pass_gstats(FitDev &F, double *red) {
  double v[2] = {0.0, 0.0};
  double mx = 0.0;
  for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt) {
    const double gi = F.g[i];
    v[0] = __builtin_fma(gi, gi, v[0]);
    v[1] = __builtin_fma(gi, F.d[i], v[1]);
    mx = fmax(mx, fabs(gi));
  }
  blk_sums2_max(v, mx, red);
  if (threadIdx.x == 0) {
    F.gg = v[0];
    F.dphi0 = v[1];
    F.gmax = mx;
  }
  __syncthreads();
}

// d = -H0 g (H0 = I, or the diagonal preconditioner) and its slope g.d.
__device__ __attribute__((always_inline)) inline void set_steepest(FitDev &F, double *red) {
  double v[1] = {0.0};
  for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt) {
    const double gi = F.g[i];
    const double di = F.precond ? -F.Dinv[i] * gi : -gi;
    F.d[i] = di;
    v[0] = __builtin_fma(gi, di, v[0]);
  }
  blk_sums<1>(v, red);
  if (threadIdx.x == 0) {
    F.dphi0 = v[0];
    fit_staged = 0;  // the LDS copy of d (if any) is stale
  }
  __syncthreads();
}

// Start a line search from (x, f, g) along d; F.gg, F.gmax and F.dphi0 = g.d
// must be current.
__device__ __attribute__((always_inline)) inline void start_ls(FitDev &F, double *red) {
  if (threadIdx.x == 0 && (F.gg == 0.0 || F.gmax <= F.gtol)) fit_stop(F, ST_GTOL);
  __syncthreads();
  if (F.status != ST_RUNNING) return;
  const double gnorm = sqrt(F.gg);
  double t1 = (F.hist_len == 0 && !F.precond) ? 1.0 / gnorm : 1.0;
  if (!(F.dphi0 < 0.0)) {
    set_steepest(F, red);
    t1 = F.precond ? 1.0 : 1.0 / gnorm;
    if (threadIdx.x == 0) F.hist_len = 0;
  }
  if (threadIdx.x == 0) {
    F.f0 = F.f;
    F.prev_t = 0.0;
    F.prev_f = F.f;
    F.prev_d = F.dphi0;
    F.t = t1;
    F.ls_evals = 0;
    F.phase = PH_BRACKET;
  }
  __syncthreads();
}

// Dinv = 1 / (diag + floor * max diag) from the last evaluation; the gauge row of
// grain N-1 stays 0.
__device__ __attribute__((always_inline)) inline void refresh_dinv(FitDev &F, double *red) {
  double mx = 0.0;
  for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt) mx = fmax(mx, F.diag[i]);
  mx = blk_max(mx, red);
  const double fl = F.diag_floor * mx;
  const int last = (F.N - 1) * F.K;
  for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt) {
    const double w = (F.gauge == 0 && i >= last) ? 0.0 : 1.0 / (F.diag[i] + fl);
    F.Dinv[i] = w;
    if (F.NK < FIT_SPLIT_MIN_NK) fit_vec[FV_W][i] = w;
  }
  __syncthreads();
}

// gYY[j][k] = y_j . Dinv y_k for every pair of the L live slots, in tiles of 4
// rows x 8 columns on or right of the diagonal block (one pass over memory and
// one 32-value block sum per tile).
__device__ __attribute__((always_inline)) inline void gram_yy(FitDev &F, const int *slot, int L, double *gYY, double *red) {
  const int M1 = F.m + 1;
  const int n = F.NK;
  const auto pY = pd_glb((const double *)F.Y);
  const auto pw = pd_glb((const double *)F.Dinv);
  for (int a0 = 0; a0 < L; a0 += 4) {
    for (int b0 = a0; b0 < L; b0 += 8) {
      int ja[4], jb[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) ja[u] = slot[min(a0 + u, L - 1)];
#pragma unroll
      for (int v = 0; v < 8; ++v) jb[v] = slot[min(b0 + v, L - 1)];
      double acc[32];
#pragma unroll
      for (int q = 0; q < 32; ++q) acc[q] = 0.0;
      for (int e = (int)threadIdx.x; e < n && (int)threadIdx.x < F.vt; e += F.vt) {
        const double w = pw[e];
        double ya[4], yb[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) ya[u] = pY[(size_t)ja[u] * n + e] * w;
#pragma unroll
        for (int v = 0; v < 8; ++v) yb[v] = pY[(size_t)jb[v] * n + e];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 8; ++v) acc[u * 8 + v] = __builtin_fma(ya[u], yb[v], acc[u * 8 + v]);
      }
      blk_sums<32>(acc, red);
      // constant indices only: a runtime bound here would move acc to scratch
      if (threadIdx.x == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 8; ++v)
            if (a0 + u < L && b0 + v < L) {
              gYY[ja[u] * M1 + jb[v]] = acc[u * 8 + v];
              gYY[jb[v] * M1 + ja[u]] = acc[u * 8 + v];
            }
      }
      __syncthreads();
    }
  }
}

// The 5 U dot products of the live slots k0 .. k0+U-1 over the elements
// e0 + tid, e0 + tid + nthr, ... < e1: S^T g, Y^T g (in the metric of H0:
// Dinv, or the identity), s_new . Y, S . y_new, y_new . Y (same metric).
template <int U>
__device__ __attribute__((always_inline)) inline void dots_accumulate(
    const FitDev &F, const int (&js)[U], const double *s, const double *y, int e0, int e1,
    int tid, int nthr, double (&acc)[5 * U]) {
  const int n = F.NK;
  const auto pS = pd_glb((const double *)F.S);
  const auto pY = pd_glb((const double *)F.Y);
  const auto pg = pd_glb((const double *)F.g);
  const auto pns = pd_glb(s);
  const auto pny = pd_glb(y);
  const auto pw = pd_glb((const double *)F.Dinv);
  const bool pre = F.precond != 0;
#pragma unroll
  for (int q = 0; q < 5 * U; ++q) acc[q] = 0.0;
  // two elements per thread at a time, all their loads issued together
  for (int e = e0 + tid; e < e1; e += 2 * nthr) {
    double gi[2], si[2], yi[2], w[2], Sj[2][U], Yj[2][U];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = e + h * nthr;
      const bool ok = i < e1;
      gi[h] = ok ? pg[i] : 0.0;
      si[h] = ok ? pns[i] : 0.0;
      yi[h] = ok ? pny[i] : 0.0;
      w[h] = (ok && pre) ? pw[i] : 1.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        Sj[h][u] = ok ? pS[(size_t)js[u] * n + i] : 0.0;
        Yj[h][u] = ok ? pY[(size_t)js[u] * n + i] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (e + h * nthr >= e1) continue;
      const double gw = pre ? gi[h] * w[h] : gi[h], yw = pre ? yi[h] * w[h] : yi[h];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc[u] = __builtin_fma(Sj[h][u], gi[h], acc[u]);
        acc[U + u] = __builtin_fma(Yj[h][u], gw, acc[U + u]);
        acc[2 * U + u] = __builtin_fma(si[h], Yj[h][u], acc[2 * U + u]);
        acc[3 * U + u] = __builtin_fma(Sj[h][u], yi[h], acc[3 * U + u]);
        acc[4 * U + u] = __builtin_fma(yw, Yj[h][u], acc[4 * U + u]);
      }
    }
  }
}

// The dot products of slot k (oldest first, ring slot jj) into the LDS copies:
// v = (S^T g, Y^T g, s_new . y_jj, s_jj . y_new, y_new . y_jj).
__device__ inline void put_slot_dots(int jj, bool stored, int put, int M1, double v0, double v1,
                                     double v2, double v3, double v4, double *Sg, double *Yg,
                                     double *gSY, double *gYY) {
  Sg[jj] = v0;
  Yg[jj] = v1;
  if (stored) {
    gSY[put * M1 + jj] = v2;
    gSY[jj * M1 + put] = v3;
    gYY[put * M1 + jj] = v4;
    gYY[jj * M1 + put] = v4;
  }
}

// v of lane k (k wave-uniform) on every lane.
__device__ inline double lane_bcast(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

// Coefficients of the compact two-loop recursion on the lanes of wave 0: alpha
// newest to oldest, then beta oldest to newest.  Lane j holds alpha_j, beta_j
// and the running sum of the terms of the pairs already done; each step
// broadcasts the finished alpha_k (beta_k) and every lane adds its term.  The
// loops are not unrolled (this code runs once per launch, so its size, not its
// instruction count, sets the time) and each step's Gram entry is loaded one
// step ahead.
__device__ __attribute__((always_inline)) inline void lbfgs_coef(
    FitDev &F, int L, int head, int M1, const int *slot, const double *rho, const double *Sg,
    const double *Yg, const double *gSY, const double *gYY, double *coef) {
  const int lane = threadIdx.x;
  const bool live = lane < L;
  const int jl = live ? slot[lane] : 0;
  const double rho_l = live ? rho[jl] : 0.0;
  const double sg_l = live ? Sg[jl] : 0.0;
  auto slot_of = [&](int k) { return head + k >= M1 ? head + k - M1 : head + k; };
  // alpha_j = rho_j (s_j.g - sum_{k>j} alpha_k s_j.y_k)
  double a = 0.0, pa = 0.0;
  double nx = L > 0 ? gSY[jl * M1 + slot_of(L - 1)] : 0.0;
  for (int k = L - 1; k >= 0; --k) {
    const double e = live ? nx : 0.0;
    if (k > 0) nx = gSY[jl * M1 + slot_of(k - 1)];
    const double ak = lane_bcast(rho_l * (sg_l - pa), k);
    if (lane == k) a = ak;
    pa = __builtin_fma(ak, e, pa);
  }
  const double gam = L > 0 ? F.gamma : 1.0;
  // y_j . q_final = y_j.g - sum_k alpha_k y_j.y_k
  double yq = live ? Yg[jl] : 0.0;
  nx = L > 0 ? gYY[jl * M1 + slot_of(0)] : 0.0;
  for (int k = 0; k < L; ++k) {
    const double e = live ? nx : 0.0;
    if (k + 1 < L) nx = gYY[jl * M1 + slot_of(k + 1)];
    yq = __builtin_fma(-lane_bcast(a, k), e, yq);
  }
  // beta_j = rho_j (gamma y_j.q_final + sum_{k<j} (alpha_k - beta_k) s_k.y_j)
  double b = 0.0, pb = 0.0;
  nx = L > 0 ? gSY[slot_of(0) * M1 + jl] : 0.0;
  for (int k = 0; k < L; ++k) {
    const double e = live ? nx : 0.0;
    if (k + 1 < L) nx = gSY[slot_of(k + 1) * M1 + jl];
    const double bk = lane_bcast(rho_l * __builtin_fma(gam, yq, pb), k);
    if (lane == k) b = bk;
    pb = __builtin_fma(lane_bcast(a, k) - bk, e, pb);
  }
  if (live) {
    coef[lane] = gam * a;            // on y_k
    coef[M1 + lane] = -(a - b);      // on s_k
  }
  if (lane == 0) coef[4 * M1] = -gam;  // on g
}

// Accept the trial point (xt, graw = gradient of f, ft); update the memory and
// its Gram matrices, form the quasi-Newton direction d = -H g (the two-loop
// recursion written through S^T g, Y^T g, S^T Y and Y^T Y) and start the next
// search.
// d = H0 (cg g + sum coef_y y) + sum coef_s s over the elements e0 + tid,
// e0 + tid + nthr, ... < e1 (written to F.d), with the partial statistics g.g,
// g.d and max |g| of those elements.  Slot k of the live pairs is ring slot
// (head + k) mod M1; coef as written by lbfgs_coef.
__device__ __attribute__((always_inline)) inline void dir_accumulate(
    const FitDev &F, int head, int L, int M1, const double *coef, int e0, int e1, int tid,
    int nthr, double (&v)[2], double &mx) {
  const int n = F.NK;
  const double cg = coef[4 * M1];
  const auto pS = pd_glb((const double *)F.S);
  const auto pY = pd_glb((const double *)F.Y);
  const auto pg = pd_glb((const double *)F.g);
  const auto pdir = pd_glb(F.d);
  const auto pw = pd_glb((const double *)F.Dinv);
  const bool pre = F.precond != 0;
  // two elements per thread at a time: their loads are issued before the stores
  for (int e = e0 + tid; e < e1; e += 2 * nthr) {
    double gi[2], w[2], dy[2], ds[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = e + h * nthr;
      gi[h] = i < e1 ? pg[i] : 0.0;
      w[h] = (i < e1 && pre) ? pw[i] : 0.0;
      // d = H0 (cg g + sum coef_y y) + sum coef_s s, H0 = Dinv or the identity
      dy[h] = cg * gi[h];
      ds[h] = 0.0;
    }
    // slots in blocks of 16: the loads of a block are issued before use
    for (int k0 = 0; k0 < L; k0 += 16) {
      double yv[2][16], sv[2][16];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = e + h * nthr;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          int j = head + min(k0 + u, L - 1);
          if (j >= M1) j -= M1;
          yv[h][u] = i < e1 ? pY[(size_t)j * n + i] : 0.0;
          sv[h][u] = i < e1 ? pS[(size_t)j * n + i] : 0.0;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (k0 + u < L) {
            dy[h] = __builtin_fma(coef[k0 + u], yv[h][u], dy[h]);
            ds[h] = __builtin_fma(coef[M1 + k0 + u], sv[h][u], ds[h]);
          }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = e + h * nthr;
      if (i >= e1) continue;
      const double di = pre ? __builtin_fma(w[h], dy[h], ds[h]) : dy[h] + ds[h];
      pdir[i] = di;
      v[0] = __builtin_fma(gi[h], gi[h], v[0]);
      v[1] = __builtin_fma(gi[h], di, v[1]);
      mx = fmax(mx, fabs(gi[h]));
    }
  }
}

// Second part of an accepted step of a multi-block map (k_fit_rec): the
// memory's dot products from the blocks' partials of k_fit_dots, the
// preconditioner's Y-Grams on a refresh, gamma, and the recursion's
// coefficients (in coef and F.coef_g, for k_fit_dir).
__device__ __attribute__((always_inline)) inline void accept_mid(
    FitDev &F, double *red, int *slot, double *coef, double *gSY, double *gYY, bool stored,
    int put, bool refresh, double sy) {
  const int M1 = F.m + 1;
  const int L = F.hist_len, head = F.hist_head;
  // slot of the k-th live pair (oldest first), kept in LDS
  for (int k = threadIdx.x; k < L; k += blockDim.x) slot[k] = (head + k) % M1;
  double *Sg = coef + 4 * M1 + 1, *Yg = Sg + M1, *rho = Yg + M1;
  for (int e = threadIdx.x; e < M1 * M1; e += blockDim.x) {
    gSY[e] = F.SY[e];
    gYY[e] = F.YY[e];
  }
  for (int e = threadIdx.x; e < M1; e += blockDim.x) rho[e] = F.rho[e];
  // the blocks' partials (5 values per live slot), added in block order
  const auto pp = pd_glb((const double *)F.part);
  for (int v = threadIdx.x; v < 5 * L; v += blockDim.x) {
    double t = 0.0;
    int c = 0;
    for (; c + 8 <= F.nchunk; c += 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = pp[(size_t)(c + u) * FIT_PART_W + v];
#pragma unroll
      for (int u = 0; u < 8; ++u) t += a[u];
    }
    for (; c < F.nchunk; ++c) t += pp[(size_t)c * FIT_PART_W + v];
    red[v] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < L; ++k)
      put_slot_dots(slot[k], stored, put, M1, red[5 * k], red[5 * k + 1], red[5 * k + 2],
                    red[5 * k + 3], red[5 * k + 4], Sg, Yg, gSY, gYY);
  __syncthreads();
  if (refresh) gram_yy(F, slot, L, gYY, red);
  if (F.precond && stored && threadIdx.x == 0) F.gamma = sy / gYY[put * M1 + put];
  __syncthreads();
  // alpha (newest to oldest) and beta (oldest to newest) on the lanes of wave 0
  if (threadIdx.x < PD_WAVE) lbfgs_coef(F, L, head, M1, slot, rho, Sg, Yg, gSY, gYY, coef);
  __syncthreads();
  for (int e = threadIdx.x; e <= 4 * M1; e += blockDim.x) F.coef_g[e] = coef[e];
  if (stored || refresh)
    for (int e = threadIdx.x; e < M1 * M1; e += blockDim.x) {
      F.SY[e] = gSY[e];
      F.YY[e] = gYY[e];
    }
}

// Last part of an accepted step of a multi-block map (k_fit_start): the
// direction's statistics from the blocks' partials of k_fit_dir, then the next
// search's start.
__device__ __attribute__((always_inline)) inline void accept_tail(FitDev &F, double *red) {
  if (threadIdx.x == 0) {
    const auto pp = pd_glb((const double *)F.part);
    double v0 = 0.0, v1 = 0.0, mx = 0.0;
    int c = 0;
    for (; c + 8 <= F.nchunk; c += 8) {
      double a[8], b[8], m[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const auto row = pp + (size_t)(c + u) * FIT_PART_W;
        a[u] = row[0];
        b[u] = row[1];
        m[u] = row[2];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v0 += a[u];
        v1 += b[u];
        mx = fmax(mx, m[u]);
      }
    }
    for (; c < F.nchunk; ++c) {
      const auto row = pp + (size_t)c * FIT_PART_W;
      v0 += row[0];
      v1 += row[1];
      mx = fmax(mx, row[2]);
    }
    F.gg = v0;
    F.dphi0 = v1;
    F.gmax = mx;
    if (F.precond) *F.want_diag = ((F.iters + 1) % F.precond) == 0 ? 1 : 0;
  }
  __syncthreads();
  start_ls(F, red);
}

// The five dot products of accept_mid for a single-block map, wave by wave:
// wave w takes the live slots k = w, w + nw, ... (US at a time) over all
// elements (UE per lane; the new vectors and the metric from LDS), adds them
// across its lanes and writes them to res[5 k .. 5 k + 4] in put_slot_dots'
// order.
template <int UE, int US>
__device__ __attribute__((always_inline)) inline void wave_slot_dots(const FitDev &F, int L,
                                                                     int head, int M1, double *res) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int n = F.NK;
  const auto pS = pd_glb((const double *)F.S);
  const auto pY = pd_glb((const double *)F.Y);
  for (int k0 = w; k0 < L; k0 += US * nw) {
    int js[US];
#pragma unroll
    for (int u = 0; u < US; ++u) {
      int j = head + min(k0 + u * nw, L - 1);
      js[u] = j >= M1 ? j - M1 : j;
    }
    double sv[US][UE], yv[US][UE];
#pragma unroll
    for (int c = 0; c < UE; ++c) {
      const int e = lane + PD_WAVE * c;
      const bool ok = e < n;
#pragma unroll
      for (int u = 0; u < US; ++u) {
        sv[u][c] = ok ? pS[(size_t)js[u] * n + e] : 0.0;
        yv[u][c] = ok ? pY[(size_t)js[u] * n + e] : 0.0;
      }
    }
    double acc[5 * US];
#pragma unroll
    for (int q = 0; q < 5 * US; ++q) acc[q] = 0.0;
#pragma unroll
    for (int c = 0; c < UE; ++c) {
      const int e = lane + PD_WAVE * c;
      const bool ok = e < n;
      const double gi = ok ? fit_vec[FV_G][e] : 0.0;
      const double si = ok ? fit_vec[FV_S][e] : 0.0;
      const double yi = ok ? fit_vec[FV_Y][e] : 0.0;
      const double wi = ok ? fit_vec[FV_W][e] : 0.0;
      const double gw = gi * wi, yw = yi * wi;
#pragma unroll
      for (int u = 0; u < US; ++u) {
        acc[u] = __builtin_fma(sv[u][c], gi, acc[u]);
        acc[US + u] = __builtin_fma(yv[u][c], gw, acc[US + u]);
        acc[2 * US + u] = __builtin_fma(si, yv[u][c], acc[2 * US + u]);
        acc[3 * US + u] = __builtin_fma(sv[u][c], yi, acc[3 * US + u]);
        acc[4 * US + u] = __builtin_fma(yw, yv[u][c], acc[4 * US + u]);
      }
    }
#pragma unroll
    for (int q = 0; q < 5 * US; ++q) acc[q] = pd_wave_sum(acc[q]);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < US; ++u) {
        const int k = k0 + u * nw;
        if (k < L)
#pragma unroll
          for (int q = 0; q < 5; ++q) res[5 * k + q] = acc[q * US + u];
      }
    }
  }
}

// An accepted step of a single-block map (everything after the new pair is
// formed): the dot products wave by wave, the recursion, the direction (its
// memory loads for the thread's first element issued before the recursion)
// and the next search's start.  x and d end in fit_vec for form_trial.
__device__ __attribute__((always_inline)) inline void accept_small(
    FitDev &F, double *red, int *slot, double *coef, double *gSY, double *gYY, bool stored,
    int put, bool refresh, double sy) {
  const int n = F.NK;
  const int M1 = F.m + 1;
  const int L = F.hist_len, head = F.hist_head;
  const int tid = threadIdx.x, bd = blockDim.x;
  double *Sg = coef + 4 * M1 + 1, *Yg = Sg + M1, *rho = Yg + M1;
  // the Gram matrices and rho: loaded here, stored to LDS once the dot
  // products' loads (issued after these) have arrived
  const int MM = M1 * M1;
  const double q0 = tid < MM ? F.SY[tid] : 0.0;
  const double q1 = tid < MM ? F.YY[tid] : 0.0;
  const double q2 = tid + bd < MM ? F.SY[tid + bd] : 0.0;
  const double q3 = tid + bd < MM ? F.YY[tid + bd] : 0.0;
  const double qr = tid < M1 ? F.rho[tid] : 0.0;
  const int E = (n + PD_WAVE - 1) / PD_WAVE;
  if (E <= 4) wave_slot_dots<4, 4>(F, L, head, M1, red);
  else if (E <= 8) wave_slot_dots<8, 2>(F, L, head, M1, red);
  else wave_slot_dots<16, 1>(F, L, head, M1, red);
  FIT_STAMP(F, 7);
  for (int k = tid; k < L; k += bd) slot[k] = (head + k) % M1;
  if (tid < MM) {
    gSY[tid] = q0;
    gYY[tid] = q1;
  }
  if (tid + bd < MM) {
    gSY[tid + bd] = q2;
    gYY[tid + bd] = q3;
  }
  for (int e = tid + 2 * bd; e < MM; e += bd) {
    gSY[e] = F.SY[e];
    gYY[e] = F.YY[e];
  }
  if (tid < M1) rho[tid] = qr;
  __syncthreads();
  // the new dot products into the Gram copies (distinct entries per slot)
  for (int k = tid; k < L; k += bd)
    put_slot_dots(slot[k], stored, put, M1, red[5 * k], red[5 * k + 1], red[5 * k + 2],
                  red[5 * k + 3], red[5 * k + 4], Sg, Yg, gSY, gYY);
  __syncthreads();
  FIT_STAMP(F, 13);
  if (refresh) gram_yy(F, slot, L, gYY, red);
  if (F.precond && stored && tid == 0) F.gamma = sy / gYY[put * M1 + put];
  // the direction's memory rows for this thread's first element, in flight
  // during the recursion
  const auto pS = pd_glb((const double *)F.S);
  const auto pY = pd_glb((const double *)F.Y);
  const bool own = tid < F.vt && tid < n;
  double yv[16], sv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    int j = head + min(u, L - 1);
    if (j >= M1) j -= M1;
    const bool ok = own && u < L;
    yv[u] = ok ? pY[(size_t)j * n + tid] : 0.0;
    sv[u] = ok ? pS[(size_t)j * n + tid] : 0.0;
  }
  FIT_STAMP(F, 14);
  __syncthreads();
  FIT_STAMP(F, 8);
  if (tid < PD_WAVE) lbfgs_coef(F, L, head, M1, slot, rho, Sg, Yg, gSY, gYY, coef);
  __syncthreads();
  FIT_STAMP(F, 9);
  if (stored || refresh)
    for (int e = tid; e < MM; e += bd) {
      F.SY[e] = gSY[e];
      F.YY[e] = gYY[e];
    }
  // d = H0 (cg g + sum coef_y y) + sum coef_s s, H0 = Dinv or the identity
  const double cg = coef[4 * M1];
  const auto pdir = pd_glb(F.d);
  double v[2] = {0.0, 0.0};
  double mx = 0.0;
  for (int i = tid; i < n && tid < F.vt; i += F.vt) {
    const double gi = fit_vec[FV_G][i];
    double dy = cg * gi, ds = 0.0;
    int k0 = 0;
    if (i == tid) {
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (u < L) {
          dy = __builtin_fma(coef[u], yv[u], dy);
          ds = __builtin_fma(coef[M1 + u], sv[u], ds);
        }
      k0 = 16;
    }
    for (; k0 < L; k0 += 16) {
      double ya[16], sa[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        int j = head + min(k0 + u, L - 1);
        if (j >= M1) j -= M1;
        ya[u] = pY[(size_t)j * n + i];
        sa[u] = pS[(size_t)j * n + i];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (k0 + u < L) {
          dy = __builtin_fma(coef[k0 + u], ya[u], dy);
          ds = __builtin_fma(coef[M1 + k0 + u], sa[u], ds);
        }
    }
    const double di = F.precond ? __builtin_fma(fit_vec[FV_W][i], dy, ds) : dy + ds;
    pdir[i] = di;
    fit_vec[FV_D][i] = di;
    v[0] = __builtin_fma(gi, gi, v[0]);
    v[1] = __builtin_fma(gi, di, v[1]);
    mx = fmax(mx, fabs(gi));
  }
  blk_sums2_max(v, mx, red);
  if (tid == 0) {
    F.gg = v[0];
    F.dphi0 = v[1];
    F.gmax = mx;
    if (F.precond) *F.want_diag = ((F.iters + 1) % F.precond) == 0 ? 1 : 0;
    fit_staged = 1;  // x (from the new pair's pass) and d are in fit_vec
  }
  __syncthreads();
  FIT_STAMP(F, 10);
  start_ls(F, red);
  FIT_STAMP(F, 11);
}

__device__ __attribute__((always_inline)) inline void accept_trial(FitDev &F, double ft, double *red, int *slots,
                                                                   double *coef, double *gSY, double *gYY) {
  const int n = F.NK;
  const int m = F.m;
  const int M1 = m + 1;  // ring slots: a candidate never overwrites a stored pair
  const int put = (F.hist_head + F.hist_len) % M1;
  double *s = F.S + (size_t)put * n;
  double *y = F.Y + (size_t)put * n;
  const double t = F.t;
  FIT_STAMP(F, 5);
  double v3[3] = {0.0, 0.0, 0.0};
  double gm = 0.0;  // largest |g| of the new iterate (traced fits)
  {
    const auto ps = pd_glb(s);
    const auto py = pd_glb(y);
    const auto px = pd_glb(F.x);
    const auto pg = pd_glb(F.g);
    const auto pd = pd_glb((const double *)F.d);
    const auto pgr = pd_glb((const double *)F.graw);
    const auto pxt = pd_glb((const double *)F.xt);
    const auto pw = pd_glb((const double *)F.Dinv);
    const bool pre = F.precond != 0;
    const bool small = !F.split;
    const bool rec = F.rec != nullptr;
    // FIT_UNROLL elements per thread at a time: every load is issued before
    // the stores (which the compiler could not otherwise move them past)
    for (int i0 = (int)threadIdx.x; i0 < n && (int)threadIdx.x < F.vt; i0 += FIT_UNROLL * F.vt) {
      double dd[FIT_UNROLL], gr[FIT_UNROLL], go[FIT_UNROLL], xx[FIT_UNROLL], ww[FIT_UNROLL];
#pragma unroll
      for (int u = 0; u < FIT_UNROLL; ++u) {
        const int i = i0 + u * F.vt;
        const bool ok = i < n;
        dd[u] = ok ? pd[i] : 0.0;
        gr[u] = ok ? pgr[i] : 0.0;
        go[u] = ok ? pg[i] : 0.0;
        xx[u] = ok ? pxt[i] : 0.0;
        ww[u] = (ok && small && pre) ? pw[i] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < FIT_UNROLL; ++u) {
        const int i = i0 + u * F.vt;
        if (i < n) {
          const double si = t * dd[u];
          const double yi = gr[u] - go[u];
          ps[i] = si;
          py[i] = yi;
          v3[0] = __builtin_fma(si, yi, v3[0]);
          v3[1] = __builtin_fma(si, si, v3[1]);
          v3[2] = __builtin_fma(yi, yi, v3[2]);
          px[i] = xx[u];
          pg[i] = gr[u];
          if (rec) gm = fmax(gm, fabs(gr[u]));
          if (small) {
            fit_vec[FV_G][i] = gr[u];
            fit_vec[FV_S][i] = si;
            fit_vec[FV_Y][i] = yi;
            fit_vec[FV_W][i] = ww[u];
            fit_vec[FV_X][i] = xx[u];
          }
        }
      }
    }
  }
  blk_sums<3>(v3, red);
  if (F.rec != nullptr) gm = blk_max(gm, red);
  FIT_STAMP(F, 6);
  const double sy = v3[0], ss = v3[1], yy = v3[2];
  const bool stored = sy > CURV_EPS * sqrt(ss) * sqrt(yy);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (stored) {
      F.rho[put] = 1.0 / sy;
      if (F.hist_len < m) F.hist_len++;
      else F.hist_head = (F.hist_head + 1) % M1;
      if (!F.precond) F.gamma = sy / yy;
    }
    F.reset_tried = 0;
    F.f = ft;
    F.iters++;
    F.clk_last = wall_clock64();
    F.evals_last = F.evals;
    if (F.rec != nullptr) {
      // (the certified evaluation at xt also counted its correct pixels)
      const int k = F.rec_base + F.iters;
      double *row = F.rec + (size_t)((k - 1) % F.rec_cap) * PD_TRACE_FIELDS;
      row[0] = (double)k;
      row[1] = (double)(F.rec_evals + F.evals);
      row[2] = -ft;
      row[3] = gm;
      row[4] = t;
      row[5] = F.cert ? (double)F.cnt_t / (double)F.n_pix : NAN;
    }
  }
  __syncthreads();
  if (F.cert) {
    // xt, now the iterate, was assigned in its own evaluation
    if (threadIdx.x == 0) {
      F.acc = (double)F.cnt_t / (double)F.n_pix;
      if ((F.iters % F.check_every) == 0 && F.acc >= F.target_acc) {
        F.clk_target = wall_clock64();
        fit_stop(F, ST_TARGET);
      } else if (F.iters >= F.max_iter) {
        fit_stop(F, ST_BUDGET);
      }
    }
    __syncthreads();
    if (F.status != ST_RUNNING) return;
  }
  if (F.iters >= F.max_iter) {
    if (threadIdx.x == 0) {
      F.phase = PH_STOP;
      *F.assign_pending = 1;
    }
    __syncthreads();
    return;
  }
  if (threadIdx.x == 0 && !F.cert && (F.iters % F.check_every) == 0) *F.assign_pending = 1;
  const bool refresh = F.precond > 0 && (F.iters % F.precond) == 0;
  if (refresh) refresh_dinv(F, red);
  if (F.split) {
    // the rest runs as k_fit_dots, k_fit_rec, k_fit_dir and k_fit_start
    if (threadIdx.x == 0) {
      F.split_phase = 1;
      F.sp_put = put;
      F.sp_stored = stored ? 1 : 0;
      F.sp_refresh = refresh ? 1 : 0;
      F.sp_sy = sy;
    }
    __syncthreads();
    return;
  }
  accept_small(F, red, slots, coef, gSY, gYY, stored, put, refresh, sy);
}

// A search ended without a strong-Wolfe point.  Fall back to (t_res > 0), or
// clear the memory and retry once, or stop.
__device__ __attribute__((always_inline)) inline void ls_fail(FitDev &F, double t_res, double *red) {
  if (t_res > 0.0) {
    if (threadIdx.x == 0) {
      F.t = t_res;
      F.phase = PH_ACCEPT_NEXT;
    }
    __syncthreads();
    return;
  }
  if (F.hist_len > 0 && !F.reset_tried) {
    set_steepest(F, red);
    if (threadIdx.x == 0) {
      F.hist_len = 0;
      F.reset_tried = 1;
    }
    __syncthreads();
    start_ls(F, red);
    return;
  }
  if (threadIdx.x == 0) fit_stop(F, ST_LSFAIL);
  __syncthreads();
}

// The trial point xt = x + t d and the evaluation input
// thc = -(log2 e / eps) (xt - mean_i xt_i) (all threads of the map's block).
// Maps with N K < FIT_SPLIT_MIN_NK keep xt in LDS for the grain means, and take
// x and d from LDS when staged (right after an accepted step).
__device__ __attribute__((always_inline)) inline void form_trial(FitDev &F, double t, double *red,
                                                                 bool staged) {
  if (F.NK < FIT_SPLIT_MIN_NK) {
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt) {
      const double xi = staged ? fit_vec[FV_X][i] : F.x[i];
      const double di = staged ? fit_vec[FV_D][i] : F.d[i];
      const double v = xi + t * di;
      F.xt[i] = v;
      fit_vec[FV_XT][i] = v;
    }
    __syncthreads();
    // column sums over the grains, wave w taking columns w, w + nw, ...
    for (int k = w; k < F.K; k += nw) {
      double sm = 0.0;
      for (int i = lane; i < F.N; i += PD_WAVE) sm += fit_vec[FV_XT][i * F.K + k];
      sm = pd_wave_sum(sm);
      if (lane == 0) red[k] = sm;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt)
      F.thc[i] = F.cscale * (fit_vec[FV_XT][i] - red[i % F.K] / (double)F.N);
    return;
  }
  const auto px = pd_glb((const double *)F.x);
  const auto pd = pd_glb((const double *)F.d);
  const auto pxt = pd_glb(F.xt);
  const auto pth = pd_glb(F.thc);
  for (int i0 = (int)threadIdx.x; i0 < F.NK && (int)threadIdx.x < F.vt; i0 += FIT_UNROLL * F.vt) {
    double a[FIT_UNROLL], b[FIT_UNROLL];
#pragma unroll
    for (int u = 0; u < FIT_UNROLL; ++u) {
      const int i = i0 + u * F.vt;
      a[u] = i < F.NK ? px[i] : 0.0;
      b[u] = i < F.NK ? pd[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < FIT_UNROLL; ++u)
      if (i0 + u * F.vt < F.NK) pxt[i0 + u * F.vt] = a[u] + t * b[u];
  }
  __syncthreads();
  // column sums over the grains, VG columns at a time (loads of a grain's row
  // clamped to its last column, so all of them are issued together)
  for (int k0 = 0; k0 < F.K; k0 += VG) {
    double sm[VG];
#pragma unroll
    for (int q = 0; q < VG; ++q) sm[q] = 0.0;
    const int cnt = min(VG, F.K - k0);
    for (int i = (int)threadIdx.x; i < F.N && (int)threadIdx.x < F.vt; i += F.vt) {
      double v[VG];
#pragma unroll
      for (int q = 0; q < VG; ++q) v[q] = pxt[(size_t)i * F.K + k0 + min(q, cnt - 1)];
#pragma unroll
      for (int q = 0; q < VG; ++q)
        if (q < cnt) sm[q] += v[q];
    }
    blk_sums<VG>(sm, red);
    for (int i = (int)threadIdx.x; i < F.N && (int)threadIdx.x < F.vt; i += F.vt) {
      double v[VG];
#pragma unroll
      for (int q = 0; q < VG; ++q) v[q] = pxt[(size_t)i * F.K + k0 + min(q, cnt - 1)];
#pragma unroll
      for (int q = 0; q < VG; ++q)
        if (q < cnt) pth[(size_t)i * F.K + k0 + q] = F.cscale * (v[q] - sm[q] / (double)F.N);
    }
  }
}

// Consume a pending accuracy check of the last accepted iterate (thread 0;
// n_correct = the assignment's count).
__device__ inline void consume_acc(FitDev &F, long long n_correct) {
  *F.assign_pending = 0;
  F.acc = (double)n_correct / (double)F.n_pix;
  if (F.acc >= F.target_acc) {
    F.status = ST_TARGET;
    *F.active = 0;
    F.clk_target = wall_clock64();
    if (F.want_diag) *F.want_diag = 0;
  } else if (F.phase == PH_STOP) {
    F.status = ST_BUDGET;
    *F.active = 0;
    if (F.want_diag) *F.want_diag = 0;
  }
}

// Shared scratch of the decision kernel.
#define HS (FIT_MAX_HISTORY + 1)
#define DEC_SHARED                                  \
  __shared__ double red[MAX_WAVES * 48 + 48];       \
  __shared__ int slots[HS];                         \
  __shared__ double coef[8 * HS];                   \
  __shared__ double gSY[HS * HS], gYY[HS * HS];     \
  __shared__ FitDev sF;                             \
  __shared__ int action;

// Start of a resumed fit.  A fit that stops at its budget has stored its last
// pair (s, y, rho) but skipped the rest of that accepted step, which the
// uninterrupted fit would have done: the preconditioner refresh due at that
// iterate (from the Hessian diagonal of this start's evaluation), the Gram
// entries of the new pair and, with the preconditioner, gamma.  So the Gram
// matrices of the live pairs are formed again here (s_j.y_k, and y_j.y_k in the
// metric of H0), gamma too with the preconditioner; then g = graw and d = -H g by
// the two-loop recursion over the stored pairs (newest to oldest, then back),
// H0 = gamma I or gamma D^-1.  Every dot product is a fixed-order block sum.
__device__ __attribute__((always_inline)) inline void resumed_direction(FitDev &F, double *red) {
  const int n = F.NK, M1 = F.m + 1, L = F.hist_len;
  __shared__ double alpha[FIT_MAX_HISTORY + 1];
  if (F.precond && (F.iters % F.precond) == 0) refresh_dinv(F, red);
  for (int a = 0; a < L; ++a) {
    const int ja = (F.hist_head + a) % M1;
    const double *sa = F.S + (size_t)ja * n, *ya = F.Y + (size_t)ja * n;
    for (int b = 0; b < L; ++b) {
      const int jb = (F.hist_head + b) % M1;
      const double *yb = F.Y + (size_t)jb * n;
      double v[2] = {0.0, 0.0};
      for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt) {
        v[0] = __builtin_fma(sa[i], yb[i], v[0]);
        v[1] = __builtin_fma(F.precond ? ya[i] * F.Dinv[i] : ya[i], yb[i], v[1]);
      }
      blk_sums<2>(v, red);
      if (threadIdx.x == 0) {
        F.SY[ja * M1 + jb] = v[0];
        F.YY[ja * M1 + jb] = v[1];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && F.precond && L > 0) {
    const int jn = (F.hist_head + L - 1) % M1;
    F.gamma = F.SY[jn * M1 + jn] / F.YY[jn * M1 + jn];
  }
  for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt) {
    F.g[i] = F.graw[i];
    F.d[i] = F.graw[i];  // q
  }
  __syncthreads();
  for (int k = L - 1; k >= 0; --k) {
    const int slot = (F.hist_head + k) % M1;
    const double *sk = F.S + (size_t)slot * n, *yk = F.Y + (size_t)slot * n;
    double v[1] = {0.0};
    for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt)
      v[0] = __builtin_fma(sk[i], F.d[i], v[0]);
    blk_sums<1>(v, red);
    const double a = F.rho[slot] * v[0];
    if (threadIdx.x == 0) alpha[k] = a;
    for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt)
      F.d[i] = __builtin_fma(-a, yk[i], F.d[i]);
    __syncthreads();
  }
  for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt)
    F.d[i] = F.gamma * (F.precond ? F.Dinv[i] * F.d[i] : F.d[i]);  // r
  __syncthreads();
  for (int k = 0; k < L; ++k) {
    const int slot = (F.hist_head + k) % M1;
    const double *sk = F.S + (size_t)slot * n, *yk = F.Y + (size_t)slot * n;
    double v[1] = {0.0};
    for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt)
      v[0] = __builtin_fma(yk[i], F.d[i], v[0]);
    blk_sums<1>(v, red);
    const double c = alpha[k] - F.rho[slot] * v[0];
    for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt)
      F.d[i] = __builtin_fma(c, sk[i], F.d[i]);
    __syncthreads();
  }
  for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt) F.d[i] = -F.d[i];
  if (threadIdx.x == 0) fit_staged = 0;
  __syncthreads();
}

__device__ __attribute__((always_inline)) inline void decide_body(FitDev &F, double *red, int *slots,
                            double *coef, double *gSY, double *gYY, int *action_p, double ft);

// grid: one block per map.  Consumes one evaluation at xt.  flags: the maps'
// activity flags, then their pending-check flags (n_maps each).
__global__ __launch_bounds__(FIT_THREADS) void k_fit_decide(FitDev *Fs, const int32_t *flags,
                                                            int n_maps) {
  DEC_SHARED
  // one round trip for both flags and the state record (which lives in LDS
  // while the kernel runs -- thread 0's line-search logic touches it many
  // times -- and is written back at the end)
  const int active = flags[blockIdx.x];
  const int pending = flags[n_maps + blockIdx.x];
  constexpr int NW = (int)(sizeof(FitDev) / sizeof(int));
  for (int w = threadIdx.x; w < NW; w += blockDim.x) ((int *)&sF)[w] = ((const int *)&Fs[blockIdx.x])[w];
  if (threadIdx.x == 0) fit_staged = 0;
  __syncthreads();
  if (active == 0) return;
  FIT_STAMP(sF, 0);
  // and one more for the objective at xt and, with a pending accuracy check of
  // the last accepted iterate (assigned in this step's objective launch), its
  // per-block counts, summed in a fixed order
  const double ft = -*sF.phi_t;
  if (sF.cert) {
    // the certified correct count of this evaluation's point xt, then clear the
    // slots that the next evaluation accumulates into
    long long c = 0;
    for (int t = threadIdx.x; t < sF.c_items; t += blockDim.x) c += sF.part_c[t];
    c = pd_wave_sum_i64(c);
    long long *cw = (long long *)red;
    if ((threadIdx.x & 63) == 0) cw[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long tot = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += cw[w];
      sF.cnt_t = tot + *sF.fb_count;
      *sF.cert_slot = 0.0;
      *sF.unc_count = 0;
      *sF.fb_count = 0;
    }
    __syncthreads();
  } else if (pending != 0) {
    long long c = 0;
    for (int t = threadIdx.x; t < sF.c_items; t += blockDim.x) c += sF.part_c[t];
    c = pd_wave_sum_i64(c);
    long long *cw = (long long *)red;
    if ((threadIdx.x & 63) == 0) cw[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long tot = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += cw[w];
      consume_acc(sF, tot);
    }
    __syncthreads();
  }
  // a map that reached the target or its budget keeps its iterate; this
  // step's evaluation is not used
  if (sF.status == ST_RUNNING) decide_body(sF, red, slots, coef, gSY, gYY, &action, ft);
  __syncthreads();
  // the next evaluation's input, while the state is at hand (an accepted step
  // on the multi-block path forms it in k_fit_start)
  if (sF.status == ST_RUNNING && sF.split_phase == 0) form_trial(sF, sF.t, red, fit_staged != 0);
  __syncthreads();
  FIT_STAMP(sF, 12);
  for (int w = threadIdx.x; w < NW; w += blockDim.x) ((int *)&Fs[blockIdx.x])[w] = ((const int *)&sF)[w];
}

__device__ __attribute__((always_inline)) inline void decide_body(FitDev &F, double *red, int *slots,
                            double *coef, double *gSY, double *gYY, int *action_p, double ft) {
  int &action = *action_p;
  const int n = F.NK;
  // gradient of f = -Phi at xt (the reduction writes it with grad_sign = -1),
  // gauge-projected, in graw
  blk_gauge(F, F.graw, red);
  FIT_STAMP(F, 1);
  if (threadIdx.x == 0) F.evals++;
  if (F.phase == PH_INIT) {
    if (F.resumed) {
      resumed_direction(F, red);
    } else {
      if (F.precond) refresh_dinv(F, red);
      for (int i = (int)threadIdx.x; i < n && (int)threadIdx.x < F.vt; i += F.vt) {
        F.g[i] = F.graw[i];
        F.d[i] = F.precond ? -F.Dinv[i] * F.graw[i] : -F.graw[i];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0 && F.precond) *F.want_diag = ((F.iters + 1) % F.precond) == 0 ? 1 : 0;
    if (threadIdx.x == 0) {
      F.f = ft;
      F.clk_first = F.clk_last = wall_clock64();
      F.evals_last = F.evals;
      if (!isfinite(ft)) {
        fit_stop(F, ST_NONFINITE);
      } else if (F.cert) {
        // the start's accuracy came with its evaluation
        F.acc = (double)F.cnt_t / (double)F.n_pix;
        if (F.acc >= F.target_acc) {
          F.clk_target = wall_clock64();
          fit_stop(F, ST_TARGET);
        } else if (F.iters >= F.max_iter) {
          fit_stop(F, ST_BUDGET);
        }
      } else {
        *F.assign_pending = 1;
        if (F.iters >= F.max_iter) F.phase = PH_STOP;
      }
    }
    __syncthreads();
    if (F.status == ST_RUNNING && F.phase == PH_INIT) {
      pass_gstats(F, red);
      start_ls(F, red);
    }
    return;
  }
  // one call site each for the accept and failure paths (they are large)
  if (F.phase == PH_ACCEPT_NEXT) {
    if (threadIdx.x == 0) action = 1;
  } else {
    double dv[1] = {0.0};
    {
      const auto pgr = pd_glb((const double *)F.graw);
      const auto pd = pd_glb((const double *)F.d);
      for (int i0 = (int)threadIdx.x; i0 < n && (int)threadIdx.x < F.vt; i0 += FIT_UNROLL * F.vt) {
        double a[FIT_UNROLL], b[FIT_UNROLL];
#pragma unroll
        for (int u = 0; u < FIT_UNROLL; ++u) {
          const int i = i0 + u * F.vt;
          a[u] = i < n ? pgr[i] : 0.0;
          b[u] = i < n ? pd[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < FIT_UNROLL; ++u)
          if (i0 + u * F.vt < n) dv[0] = __builtin_fma(a[u], b[u], dv[0]);
      }
    }
    blk_sums<1>(dv, red);
    FIT_STAMP(F, 2);
    const double dt = dv[0];
    if (threadIdx.x == 0) {
      const double t = F.t;
      // a non-finite objective counts as no sufficient decrease
      const bool too_big = !(ft <= F.f0 + LS_C1 * t * F.dphi0) || !isfinite(ft);
      F.ls_evals++;
      int act = 0;
      if (F.phase == PH_BRACKET) {
        if (too_big || (F.ls_evals > 1 && ft >= F.prev_f)) {
          F.lo_t = F.prev_t; F.lo_f = F.prev_f; F.lo_d = F.prev_d;
          F.hi_t = t; F.hi_f = ft; F.hi_d = dt;
          F.phase = PH_ZOOM;
        } else if (fabs(dt) <= -LS_C2 * F.dphi0) {
          act = 1;
        } else if (dt >= 0.0) {
          F.lo_t = t; F.lo_f = ft; F.lo_d = dt;
          F.hi_t = F.prev_t; F.hi_f = F.prev_f; F.hi_d = F.prev_d;
          F.phase = PH_ZOOM;
        } else {
          F.prev_t = t; F.prev_f = ft; F.prev_d = dt;
          F.t = 2.0 * t;
          if (F.ls_evals >= LS_MAX_EVALS) act = 3;
        }
      } else {  // PH_ZOOM
        if (too_big || ft >= F.lo_f) {
          F.hi_t = t; F.hi_f = ft; F.hi_d = dt;
        } else if (fabs(dt) <= -LS_C2 * F.dphi0) {
          act = 1;
        } else {
          if (dt * (F.hi_t - F.lo_t) >= 0.0) {
            F.hi_t = F.lo_t; F.hi_f = F.lo_f; F.hi_d = F.lo_d;
          }
          F.lo_t = t; F.lo_f = ft; F.lo_d = dt;
        }
      }
      if (act == 0 && F.phase == PH_ZOOM) {
        if (F.ls_evals >= LS_MAX_EVALS) act = 2;
        else F.t = cubic_min(F.lo_t, F.lo_f, F.lo_d, F.hi_t, F.hi_f, F.hi_d);
      }
      action = act;
    }
  }
  __syncthreads();
  FIT_STAMP(F, 3);
  const int act = action;
  if (act == 1) accept_trial(F, ft, red, slots, coef, gSY, gYY);
  else if (act >= 2) ls_fail(F, act == 2 ? F.lo_t : F.prev_t, red);
}

// ---- the multi-block path of an accepted step (maps with split set)
//
// grid of k_fit_dots / k_fit_dir: the FIT_SPLIT_CHUNK-element chunks of every
// map (chunk offsets in coff, n_maps + 1); block sums in fixed order, one
// partial row per chunk.

// The memory's dot products of this chunk (after the decision kernel's first
// part stored the new pair).
__global__ __launch_bounds__(PD_BLOCK) void k_fit_dots(FitDev *Fs, const int32_t *coff, int n_maps) {
  __shared__ double red[MAX_WAVES * 48 + 48];
  const int m = pd_find_map(coff, n_maps, blockIdx.x);
  const FitDev &F = Fs[m];
  if (*F.active == 0 || F.split_phase != 1) return;
  const int c = blockIdx.x - coff[m];
  const int e0 = c * FIT_SPLIT_CHUNK, e1 = min(F.NK, e0 + FIT_SPLIT_CHUNK);
  const int M1 = F.m + 1, L = F.hist_len, head = F.hist_head;
  const double *s = F.S + (size_t)F.sp_put * F.NK;
  const double *y = F.Y + (size_t)F.sp_put * F.NK;
  double *row = F.part + (size_t)c * FIT_PART_W;
  for (int k0 = 0; k0 < L; k0 += 8) {
    int js[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int j = head + min(k0 + u, L - 1);
      if (j >= M1) j -= M1;
      js[u] = j;
    }
    double acc[40];
    dots_accumulate<8>(F, js, s, y, e0, e1, threadIdx.x, blockDim.x, acc);
    blk_sums<40>(acc, red);
    if (threadIdx.x == 0)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + u < L)
#pragma unroll
          for (int q = 0; q < 5; ++q) row[5 * (k0 + u) + q] = acc[q * 8 + u];
  }
}

// grid: one block per map.  The memory update and the recursion from the dot
// products' partials.
__global__ __launch_bounds__(FIT_THREADS) void k_fit_rec(FitDev *Fs) {
  if (*Fs[blockIdx.x].active == 0 || Fs[blockIdx.x].split_phase != 1) return;
  __shared__ double red[MAX_WAVES * 48 + 48];
  __shared__ int slots[HS];
  __shared__ double coef[8 * HS];
  __shared__ double gSY[HS * HS], gYY[HS * HS];
  __shared__ FitDev sF;
  constexpr int NW = (int)(sizeof(FitDev) / sizeof(int));
  for (int w = threadIdx.x; w < NW; w += blockDim.x) ((int *)&sF)[w] = ((const int *)&Fs[blockIdx.x])[w];
  __syncthreads();
  accept_mid(sF, red, slots, coef, gSY, gYY, sF.sp_stored != 0, sF.sp_put, sF.sp_refresh != 0,
             sF.sp_sy);
  if (threadIdx.x == 0) sF.split_phase = 2;
  __syncthreads();
  for (int w = threadIdx.x; w < NW; w += blockDim.x) ((int *)&Fs[blockIdx.x])[w] = ((const int *)&sF)[w];
}

// The direction on this chunk and its partial statistics.
__global__ __launch_bounds__(PD_BLOCK) void k_fit_dir(FitDev *Fs, const int32_t *coff, int n_maps) {
  __shared__ double red[MAX_WAVES * 48 + 48];
  const int m = pd_find_map(coff, n_maps, blockIdx.x);
  const FitDev &F = Fs[m];
  if (*F.active == 0 || F.split_phase != 2) return;
  const int c = blockIdx.x - coff[m];
  const int e0 = c * FIT_SPLIT_CHUNK, e1 = min(F.NK, e0 + FIT_SPLIT_CHUNK);
  double v[2] = {0.0, 0.0};
  double mx = 0.0;
  dir_accumulate(F, F.hist_head, F.hist_len, F.m + 1, F.coef_g, e0, e1, threadIdx.x, blockDim.x,
                 v, mx);
  blk_sums2_max(v, mx, red);
  if (threadIdx.x == 0) {
    double *row = F.part + (size_t)c * FIT_PART_W;
    row[0] = v[0];
    row[1] = v[1];
    row[2] = mx;
  }
}

// grid: one block per map.  The search start from the direction's statistics,
// then the next trial point.
__global__ __launch_bounds__(FIT_THREADS) void k_fit_start(FitDev *Fs) {
  if (*Fs[blockIdx.x].active == 0 || Fs[blockIdx.x].split_phase != 2) return;
  __shared__ double red[MAX_WAVES * 48 + 48];
  __shared__ FitDev sF;
  constexpr int NW = (int)(sizeof(FitDev) / sizeof(int));
  for (int w = threadIdx.x; w < NW; w += blockDim.x) ((int *)&sF)[w] = ((const int *)&Fs[blockIdx.x])[w];
  __syncthreads();
  accept_tail(sF, red);
  if (threadIdx.x == 0) sF.split_phase = 0;
  __syncthreads();
  if (sF.status == ST_RUNNING) form_trial(sF, sF.t, red, false);
  __syncthreads();
  for (int w = threadIdx.x; w < NW; w += blockDim.x) ((int *)&Fs[blockIdx.x])[w] = ((const int *)&sF)[w];
}

// Start of the fit on the device clock (before any warm start work).
__global__ void k_fit_stamp(FitDev *Fs, int n_maps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_maps) Fs[p].clk_start = wall_clock64();
}

// grid: one block per map: project the start, reset the state.
__global__ __launch_bounds__(FIT_THREADS) void k_fit_init(FitDev *Fs, int zero_start) {
  FitDev &F = Fs[blockIdx.x];
  __shared__ double red[MAX_WAVES * 48 + 48];
  for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt) {
    if (zero_start) F.x[i] = 0.0;
    F.d[i] = 0.0;
  }
  __syncthreads();
  if (F.gauge == 0) {
    // a given start is moved into the gauge theta_{N-1} = 0 by the common shift
    // -theta_{N-1}, which leaves Phi and the diagram unchanged (Lemma 4.2)
    double *last = red;  // K values
    for (int k = (int)threadIdx.x; k < F.K; k += blockDim.x) last[k] = F.x[(size_t)(F.N - 1) * F.K + k];
    __syncthreads();
    for (int i = (int)threadIdx.x; i < F.NK && (int)threadIdx.x < F.vt; i += F.vt) F.x[i] -= last[i % F.K];
    __syncthreads();
  } else {
    blk_gauge(F, F.x, red);
  }
  if (threadIdx.x == 0) {
    F.status = ST_RUNNING;
    F.phase = PH_INIT;
    F.evals = F.ls_evals = F.reset_tried = 0;
    if (!F.resumed) {
      F.iters = F.hist_len = F.hist_head = 0;
      F.gamma = 1.0;
    }
    F.t = 0.0;
    F.acc = -1.0;
    F.clk_target = 0;
    F.clk_first = F.clk_last = 0;
    F.evals_last = 0;
    *F.active = 1;
    *F.assign_pending = 0;
    // the start's evaluation takes the Hessian diagonal for the first refresh (a
    // resumed fit: when its iteration count is a refresh iterate)
    if (F.want_diag) *F.want_diag = (F.precond && (!F.resumed || (F.iters % F.precond) == 0)) ? 1 : 0;
    if (F.cert) {
      *F.cert_slot = 0.0;
      *F.unc_count = 0;
      *F.fb_count = 0;
    }
  }
  // the first evaluation is at the start itself
  form_trial(F, 0.0, red, false);
}

// ------------------------------------------------------------------ host side

#define FIT_HIP(ctx, expr)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return pd_fail(ctx, PD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void pd_fit_release(pd_ctx *ctx) {
  if (ctx->fit) {
    if (ctx->fit->stream) (void)hipStreamDestroy(ctx->fit->stream);
    if (ctx->fit->phi_buf) (void)hipFree(ctx->fit->phi_buf);
    delete ctx->fit;
    ctx->fit = nullptr;
  }
}

// Objective + gradient of every running map at its trial point, and the
// pending accuracy check of its accepted iterate (amaps).
static void pd_fit_eval(pd_ctx *ctx, const EvalPlan &P, int prec, const MapDev *amaps,
                        const EvalPlan *Pdiag, hipStream_t s) {
  (void)amaps;
  if (prec == 2) {
    // matrix-core objective and gradient, then the certified assignment of xt
    pd_bf16_plan_eval(ctx, P, s, false);
    // the preconditioner's Hessian diagonal: an FP32 evaluation of the maps
    // whose refresh flag is set (its gate), at the same trial point
    if (Pdiag) pd_plan_eval(*Pdiag, true, s, false);
  } else {
    // certified assignment of xt inside the objective launch (P.cert)
    pd_plan_eval(P, true, s, false);
  }
}

// One level of the fit: L-BFGS on Phi at each map's own eps (the body of pd_fit
// without a schedule of eps).
// iter_base, eval_base (host, may be NULL): iterations and evaluations of each
// map in earlier levels of an eps schedule (the trace counts on from there)
static pd_status fit_level(pd_ctx *ctx, const pd_problem *probs, int32_t n,
                           double *const *theta_inout, const pd_fit_opts *opts,
                           pd_fit_report *reports, void *stream,
                           const int32_t *iter_base = nullptr, const int32_t *eval_base = nullptr) {
  using clk = std::chrono::steady_clock;
  const auto t_call = clk::now();
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!probs || n < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  if (!theta_inout || !opts || !reports)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_inout, opts and reports must be non-NULL");
  int prec;
  if (opts->prec == PD_FP64) prec = 0;
  else if (opts->prec == PD_FP32) prec = 1;
  else if (opts->prec == PD_BF16) prec = 2;
  else return pd_fail(ctx, PD_ERR_INVALID_ARG, "unknown precision");
  if (opts->gauge < PD_GAUGE_LAST_ZERO || opts->gauge > PD_GAUGE_NONE)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "unknown gauge");
  if (opts->init < PD_INIT_GIVEN || opts->init > PD_INIT_HEURISTIC)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "unknown init");
  if (opts->init == PD_INIT_MLP && opts->mlp == nullptr)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "PD_INIT_MLP needs opts->mlp");
  if (opts->history < 1 || opts->history > FIT_MAX_HISTORY)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "history must be in [1, 32]");
  if (opts->max_iter < 0) return pd_fail(ctx, PD_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (opts->check_every < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "check_every must be >= 1");
  if (!(opts->gtol >= 0.0)) return pd_fail(ctx, PD_ERR_INVALID_ARG, "gtol must be >= 0");
  if (opts->trace && opts->trace_cap < 1)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "trace_cap must be >= 1 with a trace");
  for (int p = 0; p < n; ++p) {
    if (!theta_inout[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_inout entry is NULL");
  }
  if (prec == 2)
    for (int p = 0; p < n; ++p)
      if (probs[p].degree > 6) return pd_fail(ctx, PD_ERR_UNSUPPORTED, "PD_BF16 supports degree <= 6");
  if (opts->resume != 0 && opts->resume != 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "resume must be 0 or 1");
  if (opts->resume) {
    if (!opts->state) return pd_fail(ctx, PD_ERR_INVALID_ARG, "resume needs the state buffers");
    if (opts->init != PD_INIT_GIVEN)
      return pd_fail(ctx, PD_ERR_INVALID_ARG, "resume needs PD_INIT_GIVEN (the iterate of the state)");
    for (int p = 0; p < n; ++p)
      if (!opts->state[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "resume: a state entry is NULL");
  }
  if (opts->precondition < 0) return pd_fail(ctx, PD_ERR_INVALID_ARG, "precondition must be >= 0");
  if (opts->precondition > 0 && opts->gauge != PD_GAUGE_LAST_ZERO)
    return pd_fail(ctx, PD_ERR_UNSUPPORTED, "the diagonal preconditioner keeps PD_GAUGE_LAST_ZERO");
  pd_status st = pd_validate(ctx, probs, n, stream);
  if (st != PD_OK) return st;
  if (opts->init == PD_INIT_MLP || opts->init == PD_INIT_HEURISTIC) {
    // warm start into the caller's buffers, then a fit from there
    st = pd_warm_start(ctx, probs, n, opts->init == PD_INIT_MLP ? opts->mlp : nullptr,
                       theta_inout, opts->prec, nullptr, stream);
    if (st != PD_OK) return st;
  }
  FIT_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->fit) ctx->fit = new FitState();
  if (!ctx->fit->stream) FIT_HIP(ctx, hipStreamCreateWithFlags(&ctx->fit->stream, hipStreamNonBlocking));
  hipStream_t s = ctx->fit->stream;
  // the fit starts after the caller's earlier work on its stream
  FIT_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));

  // ---- a saved L-BFGS state to resume from: its header must match
  const int m_hist = opts->history;
  std::vector<double> hdr((size_t)PD_FIT_STATE_HEADER * n, 0.0);
  if (opts->resume) {
    for (int p = 0; p < n; ++p)
      FIT_HIP(ctx, hipMemcpyAsync(hdr.data() + (size_t)PD_FIT_STATE_HEADER * p, opts->state[p],
                                  sizeof(double) * PD_FIT_STATE_HEADER, hipMemcpyDeviceToHost, s));
    FIT_HIP(ctx, hipStreamSynchronize(s));
    for (int p = 0; p < n; ++p) {
      const double *h = hdr.data() + (size_t)PD_FIT_STATE_HEADER * p;
      const int K = (probs[p].degree + 1) * (probs[p].degree + 2) / 2;
      const bool ok = h[0] == FIT_STATE_TAG && h[1] == probs[p].n_grains && h[2] == K &&
                      h[3] == m_hist && h[4] >= 0 && h[4] <= m_hist && h[5] >= 0 && h[5] <= m_hist &&
                      h[6] >= 0 && h[6] + opts->max_iter <= 2e9 && h[8] == opts->precondition &&
                      h[9] == (double)opts->gauge;
      if (!ok)
        return pd_fail(ctx, PD_ERR_INVALID_ARG,
                       "resume: state " + std::to_string(p) +
                           " was not written for this map, history, gauge and preconditioner");
    }
  }

  std::vector<double> hdr_iters0(n, 0.0);
  for (int p = 0; p < n; ++p) hdr_iters0[p] = hdr[(size_t)PD_FIT_STATE_HEADER * p + 6];

  // ---- layout: evaluation plan + fit state
  const int eval_prec = prec == 2 ? 2 : prec;
  EvalPlan P;
  Arena L;
  P.target_waves = pd_tuned_waves(ctx, probs, n, eval_prec);
  P.with_diag = opts->precondition > 0;
  P.onehot_pre = true;  // indicator moments once per fit
  P.sort = true;        // grains in spatial order for the far-field test
  P.cert = true;  // the accuracy of every evaluated point, certified
  pd_plan_layout(P, L, probs, n, eval_prec);
  const int m = opts->history;
  std::vector<size_t> o_vec(n);
  for (int p = 0; p < n; ++p) {
    const size_t NK = (size_t)P.maps[p].N * P.maps[p].K;
    o_vec[p] = L.take(sizeof(double) * (7 * NK + 2 * (size_t)(m + 1) * NK + (size_t)(m + 1) +
                                        2 * (size_t)(m + 1) * (m + 1) + 2 * (size_t)(m + 1)));
  }
  // multi-block passes for the large maps (PD_FIT_SPLIT_MIN overrides the size)
  int split_min = FIT_SPLIT_MIN_NK;
  if (const char *e = getenv("PD_FIT_SPLIT_MIN"))
    split_min = std::min(FIT_SPLIT_MIN_NK, std::max(1, atoi(e)));  // never above: LDS sizes
  std::vector<int32_t> coff(n + 1, 0);
  std::vector<size_t> o_split(n, 0);
  for (int p = 0; p < n; ++p) {
    const int NK = P.maps[p].N * P.maps[p].K;
    const int nch = NK >= split_min ? (NK + FIT_SPLIT_CHUNK - 1) / FIT_SPLIT_CHUNK : 0;
    coff[p + 1] = coff[p] + nch;
    if (nch) o_split[p] = L.take(sizeof(double) * (8 * (FIT_MAX_HISTORY + 1) + (size_t)nch * FIT_PART_W));
  }
  const int total_chunks = coff[n];
  const size_t o_coff = L.take(sizeof(int32_t) * (n + 1));
  const size_t o_F = L.take(sizeof(FitDev) * n);
  const size_t o_flags = L.take(sizeof(int32_t) * 3 * n);
  const size_t o_phi = L.take(sizeof(double) * n);
  const size_t o_nc = L.take(sizeof(int64_t) * n);
  const size_t o_amaps = L.take(sizeof(MapDev) * n);
  // BF16 with the preconditioner: an FP32 plan for the Hessian diagonal, gated
  // by each map's refresh flag (its gradient and objective go to scratch)
  const bool diag_plan = prec == 2 && opts->precondition > 0;
  EvalPlan P2;
  size_t o_phi2 = 0;
  std::vector<size_t> o_g2(n);
  if (diag_plan) {
    P2.target_waves = pd_tuned_waves(ctx, probs, n, 1);
    P2.with_diag = true;
    pd_plan_layout(P2, L, probs, n, 1);
    o_phi2 = L.take(sizeof(double) * n);
    for (int p = 0; p < n; ++p) o_g2[p] = L.take(sizeof(double) * (size_t)P2.maps[p].N * P2.maps[p].K);
  }
  st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;
  char *base = ctx->ws;
  std::vector<FitDev> F(n);
  std::vector<double *> xt(n), graw(n);
  int32_t *flags = (int32_t *)(base + o_flags);
  double *phi_t = (double *)(base + o_phi);
  int64_t *nc = (int64_t *)(base + o_nc);
  for (int p = 0; p < n; ++p) {
    const MapDev &M = P.maps[p];
    const size_t NK = (size_t)M.N * M.K;
    double *v = (double *)(base + o_vec[p]);
    FitDev &f = F[p];
    memset(&f, 0, sizeof(FitDev));
    f.N = M.N;
    f.K = M.K;
    f.NK = (int32_t)NK;
    f.m = m;
    f.max_iter = opts->max_iter;
    f.check_every = opts->check_every;
    f.gauge = (int)opts->gauge;
    f.vt = std::min(FIT_THREADS, std::max(64, ((int)NK + 63) / 64 * 64));
    f.n_pix = (int64_t)M.H * M.W;
    f.target_acc = opts->target_acc;
    f.gtol = opts->gtol;
    f.x = v;
    f.g = v + NK;
    f.d = v + 2 * NK;
    f.xt = v + 3 * NK;
    f.graw = v + 4 * NK;
    f.S = v + 5 * NK;
    f.Y = f.S + (size_t)(m + 1) * NK;
    f.rho = f.Y + (size_t)(m + 1) * NK;
    f.SY = f.rho + (m + 1);
    f.YY = f.SY + (size_t)(m + 1) * (m + 1);
    f.Sg = f.YY + (size_t)(m + 1) * (m + 1);
    f.Yg = f.Sg + (m + 1);
    f.Dinv = f.Yg + (m + 1);
    f.diag = f.Dinv + NK;
    f.precond = opts->precondition;
    f.want_diag = flags + 2 * n + p;
    f.diag_floor = 1e-6;
    f.phi_t = phi_t + p;
    f.cscale = -PD_LOG2E / M.eps;
    f.cert = P.cert ? 1 : 0;
    // per-wave counts of the certified objective (on the BF16 path those of
    // k16_lse or of its FP64 fallback k16_recert, the rest zeroed)
    f.c_items = P.cert ? (prec == 2 ? std::max(M.a_items, 4 * M.a16_items) : M.a_items)
                       : M.a_items / PD_WAVES_PER_BLOCK;
    f.nchunk = coff[p + 1] - coff[p];
    f.split = f.nchunk > 0 ? 1 : 0;
    if (f.split) {
      f.coef_g = (double *)(base + o_split[p]);
      f.part = f.coef_g + 8 * (FIT_MAX_HISTORY + 1);
    }
    f.active = flags + p;
    f.assign_pending = flags + n + p;
    if (opts->resume) {
      const double *h = hdr.data() + (size_t)PD_FIT_STATE_HEADER * p;
      f.resumed = 1;
      f.hist_len = (int32_t)h[4];
      f.hist_head = (int32_t)h[5];
      f.iters = (int32_t)h[6];
      f.gamma = h[7];
      f.max_iter = f.iters + opts->max_iter;
    }
    f.rec = opts->trace ? opts->trace[p] : nullptr;
    f.rec_cap = opts->trace ? opts->trace_cap : 1;
    f.rec_base = iter_base ? iter_base[p] : 0;
    f.rec_evals = eval_base ? eval_base[p] : 0;
    xt[p] = f.xt;
    graw[p] = f.graw;
  }
  pd_plan_bind(P, base, xt.data(), phi_t, graw.data(), nullptr, nullptr);
  for (int p = 0; p < n; ++p) {
    F[p].thc = P.maps[p].thc;
    F[p].part_c = P.maps[p].part_c;
    F[p].cert_slot = P.maps[p].cert;
    F[p].unc_count = P.maps[p].unc_count;
    F[p].fb_count = P.maps[p].fb_count;
  }
  for (int p = 0; p < n; ++p) {
    P.maps[p].gate = flags + p;
    P.maps[p].grad_sign = -1.0;  // the evaluation returns the gradient of f = -Phi
  }
  if (opts->precondition > 0)
    for (int p = 0; p < n; ++p) {
      P.maps[p].diag = (double *)F[p].diag;
      P.maps[p].want_diag = F[p].want_diag;
    }
  const EvalPlan *Pd = nullptr;
  if (diag_plan) {
    std::vector<double *> g2(n);
    for (int p = 0; p < n; ++p) g2[p] = (double *)(base + o_g2[p]);
    pd_plan_bind(P2, base, xt.data(), (double *)(base + o_phi2), g2.data(), nullptr, nullptr);
    for (int p = 0; p < n; ++p) {
      P2.maps[p].thc = P.maps[p].thc;        // the trial point's logit input
      P2.maps[p].gate = F[p].want_diag;      // only maps that refresh this step
      P2.maps[p].diag = (double *)F[p].diag;
      P2.maps[p].want_diag = F[p].want_diag;
    }
    Pd = &P2;
  }
  // assignment view of the same maps: theta = x, gate = assign_pending
  std::vector<MapDev> amaps = P.maps;
  for (int p = 0; p < n; ++p) {
    amaps[p].theta = F[p].x;
    amaps[p].n_correct = nc + p;
    amaps[p].labels_out = nullptr;
    amaps[p].gate = flags + n + p;
  }
  MapDev *d_amaps = (MapDev *)(base + o_amaps);
  FitDev *dF = (FitDev *)(base + o_F);
  int32_t *d_coff = (int32_t *)(base + o_coff);
#ifdef PD_FIT_TRACE
  uint64_t *trace_buf = nullptr;
  FIT_HIP(ctx, hipMalloc((void **)&trace_buf, sizeof(uint64_t) * 256 * 16 * n));
  FIT_HIP(ctx, hipMemsetAsync(trace_buf, 0, sizeof(uint64_t) * 256 * 16 * n, s));
  for (int p = 0; p < n; ++p) F[p].trace = trace_buf + (size_t)p * 256 * 16;
#endif
  FIT_HIP(ctx, pd_plan_upload(ctx, P, s));
  if (diag_plan) FIT_HIP(ctx, pd_plan_upload(ctx, P2, s));
  FIT_HIP(ctx, hipMemcpyAsync(d_amaps, amaps.data(), sizeof(MapDev) * n, hipMemcpyHostToDevice, s));
  FIT_HIP(ctx, hipMemcpyAsync(dF, F.data(), sizeof(FitDev) * n, hipMemcpyHostToDevice, s));
  FIT_HIP(ctx, hipMemcpyAsync(d_coff, coff.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
  const bool zero_start = opts->init == PD_INIT_ZERO;
  if (!zero_start)
    for (int p = 0; p < n; ++p)
      FIT_HIP(ctx, hipMemcpyAsync(F[p].x, theta_inout[p], sizeof(double) * F[p].NK,
                                  hipMemcpyDeviceToDevice, s));
  if (opts->resume)
    for (int p = 0; p < n; ++p) {
      const size_t NK = (size_t)F[p].NK;
      FIT_HIP(ctx, hipMemcpyAsync(F[p].S, opts->state[p] + PD_FIT_STATE_HEADER,
                                  sizeof(double) * fit_state_ring(NK, m), hipMemcpyDeviceToDevice, s));
      FIT_HIP(ctx, hipMemcpyAsync(F[p].Dinv, opts->state[p] + PD_FIT_STATE_HEADER + fit_state_ring(NK, m),
                                  sizeof(double) * NK, hipMemcpyDeviceToDevice, s));
    }
  const auto t_stamp = clk::now();
  k_fit_stamp<<<(n + 255) / 256, 256, 0, s>>>(dF, n);
  pd_plan_tables(P, s);
  pd_plan_onehot(P, s);
  if (diag_plan) pd_plan_tables(P2, s);
  // block size: the largest per-map thread count (about 4 elements per thread)
  int vt = 64;
  for (int p = 0; p < n; ++p) vt = std::max(vt, F[p].vt);
  k_fit_init<<<n, vt, 0, s>>>(dF, zero_start ? 1 : 0);
  FIT_HIP(ctx, hipGetLastError());

  // ---- FIT_GRAPH_STEPS steps, captured as one graph (a graph launch has a
  // fixed cost at its boundary; the steps after a map stops are gated off)
  auto step = [&](hipStream_t ss) {
    pd_fit_eval(ctx, P, eval_prec, d_amaps, Pd, ss);
    k_fit_decide<<<n, vt, 0, ss>>>(dF, flags, n);
    if (total_chunks > 0) {
      k_fit_dots<<<total_chunks, PD_BLOCK, 0, ss>>>(dF, d_coff, n);
      k_fit_rec<<<n, vt, 0, ss>>>(dF);
      k_fit_dir<<<total_chunks, PD_BLOCK, 0, ss>>>(dF, d_coff, n);
      k_fit_start<<<n, vt, 0, ss>>>(dF);
    }
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  FIT_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < FIT_GRAPH_STEPS; ++k) step(s);
  hipError_t ce = hipStreamEndCapture(s, &graph);
  if (ce != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ce != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return pd_fail(ctx, PD_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ce));
  }
  // ---- replay until every map has stopped
  int32_t *h_flags = nullptr;
  FIT_HIP(ctx, hipHostMalloc((void **)&h_flags, sizeof(int32_t) * n, hipHostMallocDefault));
  const long long max_steps = (long long)(opts->max_iter + 2) * (2 * LS_MAX_EVALS + 4) + 8;
  long long steps = 0;
  int poll = 1;
  hipError_t le = hipSuccess;
  while (steps < max_steps) {
    for (int k = 0; k < poll && le == hipSuccess; ++k, steps += FIT_GRAPH_STEPS)
      le = hipGraphLaunch(exec, s);
    if (le != hipSuccess) break;
    le = hipMemcpyAsync(h_flags, flags, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s);
    if (le != hipSuccess) break;
    le = hipStreamSynchronize(s);
    if (le != hipSuccess) break;
    bool any = false;
    for (int p = 0; p < n; ++p) any |= h_flags[p] != 0;
    if (!any) break;
    if (poll * FIT_GRAPH_STEPS < 16) poll *= 2;
  }
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  (void)hipHostFree(h_flags);
  if (le != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, std::string("fit loop: ") + hipGetErrorString(le));
  // ---- final accuracy of every map and the results
  std::vector<MapDev> fin = amaps;
  for (int p = 0; p < n; ++p) fin[p].gate = nullptr;
  FIT_HIP(ctx, hipMemcpyAsync(d_amaps, fin.data(), sizeof(MapDev) * n, hipMemcpyHostToDevice, s));
  pd_launch_assign(P.dmax, d_amaps, P.d_offA, n, P.offA[n], true, s);
  std::vector<int64_t> h_nc(n);
  FIT_HIP(ctx, hipMemcpyAsync(h_nc.data(), nc, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
  FIT_HIP(ctx, hipMemcpyAsync(F.data(), dF, sizeof(FitDev) * n, hipMemcpyDeviceToHost, s));
  for (int p = 0; p < n; ++p)
    FIT_HIP(ctx, hipMemcpyAsync(theta_inout[p], F[p].x, sizeof(double) * F[p].NK,
                                hipMemcpyDeviceToDevice, s));
  FIT_HIP(ctx, hipStreamSynchronize(s));
  const auto t_end = clk::now();
  // ---- the L-BFGS state of every map, for a later resume
  if (opts->state) {
    for (int p = 0; p < n; ++p) {
      if (!opts->state[p]) continue;
      const FitDev &f = F[p];
      double *h = hdr.data() + (size_t)PD_FIT_STATE_HEADER * p;
      for (int k = 0; k < PD_FIT_STATE_HEADER; ++k) h[k] = 0.0;
      h[0] = FIT_STATE_TAG;
      h[1] = f.N;
      h[2] = f.K;
      h[3] = f.m;
      h[4] = f.hist_len;
      h[5] = f.hist_head;
      h[6] = f.iters;
      h[7] = f.gamma;
      h[8] = f.precond;
      h[9] = f.gauge;
      const size_t NK = (size_t)f.NK;
      FIT_HIP(ctx, hipMemcpyAsync(opts->state[p], h, sizeof(double) * PD_FIT_STATE_HEADER,
                                  hipMemcpyHostToDevice, s));
      FIT_HIP(ctx, hipMemcpyAsync(opts->state[p] + PD_FIT_STATE_HEADER, f.S,
                                  sizeof(double) * fit_state_ring(NK, f.m), hipMemcpyDeviceToDevice, s));
      FIT_HIP(ctx, hipMemcpyAsync(opts->state[p] + PD_FIT_STATE_HEADER + fit_state_ring(NK, f.m), f.Dinv,
                                  sizeof(double) * NK, hipMemcpyDeviceToDevice, s));
    }
    FIT_HIP(ctx, hipStreamSynchronize(s));
  }
#ifdef PD_FIT_TRACE
  if (const char *path = getenv("PD_FIT_TRACE_OUT")) {
    std::vector<uint64_t> h((size_t)256 * 16 * n);
    (void)hipMemcpy(h.data(), trace_buf, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost);
    if (FILE *fp = fopen(path, "wb")) {
      fwrite(h.data(), sizeof(uint64_t), h.size(), fp);
      fclose(fp);
    }
  }
  (void)hipFree(trace_buf);
#endif
  int rate_khz = 0;
  (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device);
  const double host_setup = std::chrono::duration<double>(t_stamp - t_call).count();
  for (int p = 0; p < n; ++p) {
    pd_fit_report &r = reports[p];
    const FitDev &f = F[p];
    r.status = f.status == ST_RUNNING ? ST_BUDGET : f.status;
    r.iters = f.iters - (opts->resume ? (int32_t)hdr_iters0[p] : 0);
    r.evals = f.evals;
    r.phi = -f.f;
    r.acc = (double)h_nc[p] / (double)f.n_pix;
    r.seconds_total = std::chrono::duration<double>(t_end - t_call).count();
    r.seconds_iterating = rate_khz > 0 && f.clk_last >= f.clk_first
                              ? (double)(f.clk_last - f.clk_first) / ((double)rate_khz * 1e3)
                              : 0.0;
    r.evals_iterating = f.evals_last > 0 ? f.evals_last - 1 : 0;
    r.seconds_to_target = -1.0;
    // host set-up before the first device work, plus device time to the target
    if (f.status == ST_TARGET && rate_khz > 0 && f.clk_target >= f.clk_start)
      r.seconds_to_target =
          host_setup + (double)(f.clk_target - f.clk_start) / ((double)rate_khz * 1e3);
    // a stop (gradient tolerance, failed search) at an iterate whose accuracy
    // check was still pending: the accuracy test comes first
    if (r.status != ST_TARGET && r.acc >= opts->target_acc) {
      r.status = ST_TARGET;
      r.seconds_to_target = r.seconds_total;
    }
  }
  return PD_OK;
}

// The fit with an optional schedule of eps (annealing): levels
// eps_k = eps * anneal_factor^(S - k), k = 0 .. S = anneal_levels, each level a
// fit_level call from the previous level's theta with a fresh L-BFGS memory (the
// curvature of Phi_eps scales with 1/eps^2).  Level k < S has the budget
// min(anneal_iters, max_iter - k anneal_iters) iterations, the last level
// max_iter - S anneal_iters (budgets by the schedule, whatever a level used).
// F_theta does not depend on eps (Lemma 4.1), so a map that reaches the target
// accuracy at any level stops there (Err-aligned stopping); the other maps go on
// to the next level, in one batched call.
extern "C" pd_status pd_fit(pd_ctx *ctx, const pd_problem *probs, int32_t n,
                            double *const *theta_inout, const pd_fit_opts *opts,
                            pd_fit_report *reports, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!probs || n < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  if (!theta_inout || !opts || !reports)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_inout, opts and reports must be non-NULL");
  if (opts->anneal_levels < 0 || opts->anneal_levels > 30)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "anneal_levels must be in [0, 30]");
  if (opts->anneal_levels == 0) return fit_level(ctx, probs, n, theta_inout, opts, reports, stream);
  if (opts->state || opts->resume)
    return pd_fail(ctx, PD_ERR_UNSUPPORTED, "the L-BFGS state is not kept across an eps schedule");
  if (!(opts->anneal_factor > 1.0) || !std::isfinite(opts->anneal_factor))
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "anneal_factor must be finite and > 1");
  if (opts->anneal_iters < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "anneal_iters must be >= 1");
  if (opts->max_iter < 0) return pd_fail(ctx, PD_ERR_INVALID_ARG, "max_iter must be >= 0");
  using clk = std::chrono::steady_clock;
  const auto t_call = clk::now();
  const int S = opts->anneal_levels;
  std::vector<int> live(n), last_level(n, 0);
  for (int p = 0; p < n; ++p) live[p] = p;
  std::vector<double> before(n, 0.0);  // seconds of the earlier levels, per map
  for (int p = 0; p < n; ++p) {
    reports[p] = pd_fit_report{};
    reports[p].status = ST_BUDGET;
    reports[p].seconds_to_target = -1.0;
  }
  for (int k = 0; k <= S && !live.empty(); ++k) {
    const long long spent = (long long)k * opts->anneal_iters;
    const long long left = std::max(0LL, (long long)opts->max_iter - spent);
    const int budget = (int)(k == S ? left : std::min<long long>(opts->anneal_iters, left));
    if (budget == 0 && k < S) break;  // the budget ends inside the schedule
    const double f = std::pow(opts->anneal_factor, (double)(S - k));
    const int nl = (int)live.size();
    std::vector<pd_problem> pk(nl);
    std::vector<double *> tk(nl);
    for (int q = 0; q < nl; ++q) {
      pk[q] = probs[live[q]];
      pk[q].eps = probs[live[q]].eps * f;
      tk[q] = theta_inout[live[q]];
    }
    pd_fit_opts ok = *opts;
    ok.anneal_levels = 0;
    ok.max_iter = budget;
    if (k > 0) ok.init = PD_INIT_GIVEN;  // from the last level's theta
    std::vector<double *> trk(nl, nullptr);
    std::vector<int32_t> base(nl), ebase(nl);
    for (int q = 0; q < nl; ++q) {
      if (opts->trace) trk[q] = opts->trace[live[q]];
      base[q] = reports[live[q]].iters;
      ebase[q] = reports[live[q]].evals;
    }
    ok.trace = opts->trace ? trk.data() : nullptr;
    std::vector<pd_fit_report> rk(nl);
    const pd_status st = fit_level(ctx, pk.data(), nl, tk.data(), &ok, rk.data(), stream,
                                   base.data(), ebase.data());
    if (st != PD_OK) return st;
    std::vector<int> next;
    for (int q = 0; q < nl; ++q) {
      const int p = live[q];
      pd_fit_report &r = reports[p];
      const pd_fit_report &x = rk[q];
      r.status = x.status == ST_TARGET || x.status == ST_NONFINITE || k == S ? x.status : ST_BUDGET;
      r.iters += x.iters;
      r.evals += x.evals;
      r.phi = x.phi;
      r.acc = x.acc;
      r.seconds_iterating += x.seconds_iterating;
      r.evals_iterating += x.evals_iterating;
      if (x.status == ST_TARGET && x.seconds_to_target >= 0.0)
        r.seconds_to_target = before[p] + x.seconds_to_target;
      before[p] += x.seconds_total;
      last_level[p] = k;
      if (x.status != ST_TARGET && x.status != ST_NONFINITE) next.push_back(p);
    }
    live.swap(next);
  }
  // phi at each map's own eps for the maps that stopped above the last level
  std::vector<int> redo;
  for (int p = 0; p < n; ++p)
    if (last_level[p] != S) redo.push_back(p);
  if (!redo.empty()) {
    const int nr = (int)redo.size();
    std::vector<pd_problem> pr(nr);
    std::vector<const double *> th(nr);
    for (int q = 0; q < nr; ++q) {
      pr[q] = probs[redo[q]];
      th[q] = theta_inout[redo[q]];
    }
    if (!ctx->fit) ctx->fit = new FitState();
    if ((int)ctx->fit->phi_cap < nr) {
      if (ctx->fit->phi_buf) (void)hipFree(ctx->fit->phi_buf);
      ctx->fit->phi_buf = nullptr;
      ctx->fit->phi_cap = 0;
      FIT_HIP(ctx, hipMalloc((void **)&ctx->fit->phi_buf, sizeof(double) * nr));
      ctx->fit->phi_cap = nr;
    }
    const pd_status st =
        pd_objective_grad(ctx, pr.data(), nr, th.data(), ctx->fit->phi_buf, nullptr, PD_FP64, stream);
    if (st != PD_OK) return st;
    std::vector<double> ph(nr);
    FIT_HIP(ctx, hipMemcpyAsync(ph.data(), ctx->fit->phi_buf, sizeof(double) * nr,
                                hipMemcpyDeviceToHost, (hipStream_t)stream));
    FIT_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    for (int q = 0; q < nr; ++q) reports[redo[q]].phi = ph[q];
  }
  const double total = std::chrono::duration<double>(clk::now() - t_call).count();
  for (int p = 0; p < n; ++p) reports[p].seconds_total = total;
  return PD_OK;
}
