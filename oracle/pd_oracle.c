/*
 * pd_oracle.c -- plain FP64 CPU oracle for Legendre polynomial diagrams.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no source,
 * header, table or helper with the GPU library, and it is deliberately slow and
 * literal: every quantity is the paper's definition written out, in IEEE binary64
 * with round-to-nearest, no fast-math, no FMA contraction except the explicit
 * fma() calls named below.
 *
 * Paper: Bourne, Buze, Gallouet, Merigot, "Polynomial diagrams for
 * microstructure modelling" (arXiv 2605.20816).
 *
 * Conventions fixed where the paper leaves a choice (each is listed with its
 * reason in the design notes):
 *   - pixel (r, c) of an H x W map has row-major index j = r*W + c; its centre is
 *     x1 = (2c + 1 - W)/W (column axis), x2 = (2r + 1 - H)/H (row axis);
 *   - grains and labels are 0-based, 0..N-1;
 *   - multi-indices alpha = (a, b) of total degree k = a + b are ordered by k,
 *     then by b ascending: idx(a, b) = k(k+1)/2 + b  (so d = 1 gives 1, x, y);
 *   - the score of grain i is accumulated as f = theta_i0, then
 *     f = fma(theta_ia, psi_a, f) for a = 1..K-1 in index order.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Section 3.1: K_d = |A_d| = (d+1)(d+2)/2 multi-indices of total degree <= d. */
int orc_num_features(int d) { return (d + 1) * (d + 2) / 2; }

/* Section 3.1 (ordering "fixed once and for all"): degree-graded, then alpha_2
   ascending.  Writes the exponent pairs (a[k], b[k]) for k < K_d. */
void orc_multi_index(int d, int *a_out, int *b_out) {
  int idx = 0;
  for (int k = 0; k <= d; ++k)
    for (int b = 0; b <= k; ++b) {
      a_out[idx] = k - b;
      b_out[idx] = b;
      ++idx;
    }
}

/* Section 2.1: cell-centred pixels of [-1,1]^2.  For len = 2M this is
   -1 + (idx + 1/2)/M exactly; other lengths rescale the axis (Section 3.3). */
double orc_coord(int idx, int len) {
  return (double)(2 * idx + 1 - len) / (double)len;
}

/* Section 3.3: Legendre polynomials with P_0 = 1, P_1 = t and
   (m+1) P_{m+1} = (2m+1) t P_m - m P_{m-1}. */
void orc_legendre(double t, int d, double *P) {
  P[0] = 1.0;
  if (d >= 1) P[1] = t;
  for (int m = 1; m < d; ++m) {
    double a = (double)(2 * m + 1) * t;
    double b = (double)m * P[m - 1];
    P[m + 1] = fma(a, P[m], -b) / (double)(m + 1);
  }
}

/* Legendre table of one axis: out[a*len + idx] = P_a(coord(idx, len)). */
static void axis_table(int len, int d, double *out) {
  double P[16];
  for (int i = 0; i < len; ++i) {
    orc_legendre(orc_coord(i, len), d, P);
    for (int a = 0; a <= d; ++a) out[(size_t)a * len + i] = P[a];
  }
}

/* Section 3.3, design matrix eta_L(Omega): out[alpha*n + j] = P_a(x1_j) P_b(x2_j). */
void orc_features(int H, int W, int d, double *out) {
  int K = orc_num_features(d);
  int A[64], B[64];
  orc_multi_index(d, A, B);
  double *tx = (double *)malloc(sizeof(double) * (size_t)(d + 1) * W);
  double *ty = (double *)malloc(sizeof(double) * (size_t)(d + 1) * H);
  axis_table(W, d, tx);
  axis_table(H, d, ty);
  size_t n = (size_t)H * W;
  for (int k = 0; k < K; ++k)
    for (int r = 0; r < H; ++r)
      for (int c = 0; c < W; ++c)
        out[(size_t)k * n + (size_t)r * W + c] =
            tx[(size_t)A[k] * W + c] * ty[(size_t)B[k] * H + r];
  free(tx);
  free(ty);
}

/* psi(x) for one pixel into psi[0..K-1]. */
static void pixel_features(int r, int c, int H, int W, int d, const int *A,
                           const int *B, double *psi) {
  double Px[16], Py[16];
  orc_legendre(orc_coord(c, W), d, Px);
  orc_legendre(orc_coord(r, H), d, Py);
  int K = orc_num_features(d);
  for (int k = 0; k < K; ++k) psi[k] = Px[A[k]] * Py[B[k]];
}

/* Section 2.3 (linear parametrisation): h(theta_i, x) = theta_i . eta(x),
   accumulated in index order with one fma per term (psi_0 = 1 exactly). */
static double score(const double *th, const double *psi, int K) {
  double f = th[0];
  for (int k = 1; k < K; ++k) f = fma(th[k], psi[k], f);
  return f;
}

/* Neumaier's compensated summation: s + c carries the running total. */
typedef struct {
  double s, c;
} csum;
static inline void cs_add(csum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}
static inline double cs_val(const csum *a) { return a->s + a->c; }

/* Section 2.1 induced map F_theta with the smallest-index tie-break of the
   minimisation-diagram cells, and the accuracy Acc^G of Section 2.2, over the
   pixel rows [r0, r1) of the H x W map (coordinates of the whole map).
   theta: N x K row-major.  labels may be NULL (then n_correct is 0).
   out[j] = F_theta(x_j) for the pixels j of those rows (indices of the whole
   map), or -1 if any score of x_j is NaN.  Returns the number of pixels with a
   NaN score. */
int64_t orc_assign_rows(int H, int W, int N, int d, const double *theta,
                        const int32_t *labels, int r0, int r1, int32_t *out,
                        int64_t *n_correct) {
  int K = orc_num_features(d);
  int A[64], B[64];
  orc_multi_index(d, A, B);
  int64_t correct = 0, nan_count = 0;
#pragma omp parallel for schedule(static) reduction(+ : correct, nan_count)
  for (int r = r0; r < r1; ++r) {
    double psi[64];
    for (int c = 0; c < W; ++c) {
      pixel_features(r, c, H, W, d, A, B, psi);
      int best = 0;
      double fbest = score(theta, psi, K);
      int bad = isnan(fbest);
      for (int i = 1; i < N; ++i) {
        double f = score(theta + (size_t)i * K, psi, K);
        if (isnan(f)) bad = 1;
        if (f < fbest) {
          fbest = f;
          best = i;
        }
      }
      size_t j = (size_t)r * W + c;
      int lab = bad ? -1 : best;
      if (out) out[j] = lab;
      if (bad) nan_count++;
      if (labels && lab == labels[j]) correct++;
    }
  }
  if (n_correct) *n_correct = correct;
  return nan_count;
}

/* F_theta and Acc^G over the whole map. */
int64_t orc_assign(int H, int W, int N, int d, const double *theta,
                   const int32_t *labels, int32_t *out, int64_t *n_correct) {
  return orc_assign_rows(H, W, N, d, theta, labels, 0, H, out, n_correct);
}

/* Per-pixel terms of Section 2.3 / Section 4 (eq:Phi):
   s_i = -h_i/eps, m = max_i s_i, S = sum_i exp(s_i - m) (ascending i),
   lse = m + log S, ell = s_G - lse = log p^eps_G(x).
   Fills s[0..N-1] and returns ell; *lse_out receives lse. */
static double pixel_terms(const double *theta, const double *psi, int N, int K,
                          double eps, int g, double *s, double *lse_out) {
  double m = -INFINITY;
  for (int i = 0; i < N; ++i) {
    s[i] = -score(theta + (size_t)i * K, psi, K) / eps;
    if (s[i] > m) m = s[i];
  }
  double S = 0.0;
  for (int i = 0; i < N; ++i) S += exp(s[i] - m);
  double lse = m + log(S);
  *lse_out = lse;
  return s[g] - lse;
}

#define ROWS_PER_BLOCK 8

/* Objective Phi^G_eps of eq:Phi (the mean log-likelihood, maximised) and its
   gradient, eq:grad of Proposition 4.4:
     grad_i = -(1/(eps n)) sum_x (delta_{i,G(x)} - p_i(x)) eta(x).
   theta: N x K row-major; labels: n values in [0, N); grad: N x K or NULL.
   Sums are compensated; row blocks are combined in a fixed order so the result
   does not depend on the thread count. */
double orc_objective_grad(int H, int W, int N, int d, double eps,
                          const double *theta, const int32_t *labels,
                          double *grad) {
  int K = orc_num_features(d);
  int A[64], B[64];
  orc_multi_index(d, A, B);
  int nblk = (H + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
  size_t NK = (size_t)N * K;
  csum *lpart = (csum *)calloc((size_t)nblk, sizeof(csum));
  csum *gpart = grad ? (csum *)calloc((size_t)nblk * NK, sizeof(csum)) : NULL;
#pragma omp parallel
  {
    double *s = (double *)malloc(sizeof(double) * (size_t)N);
    double psi[64];
#pragma omp for schedule(dynamic, 1)
    for (int blk = 0; blk < nblk; ++blk) {
      csum lsum = {0.0, 0.0};
      csum *gp = gpart ? gpart + (size_t)blk * NK : NULL;
      int r1 = (blk + 1) * ROWS_PER_BLOCK;
      if (r1 > H) r1 = H;
      for (int r = blk * ROWS_PER_BLOCK; r < r1; ++r)
        for (int c = 0; c < W; ++c) {
          size_t j = (size_t)r * W + c;
          int g = labels[j];
          pixel_features(r, c, H, W, d, A, B, psi);
          double lse;
          double ell = pixel_terms(theta, psi, N, K, eps, g, s, &lse);
          cs_add(&lsum, ell);
          if (gp) {
            for (int i = 0; i < N; ++i) {
              double p = exp(s[i] - lse);
              double w = (i == g ? 1.0 : 0.0) - p;
              for (int k = 0; k < K; ++k) cs_add(&gp[(size_t)i * K + k], w * psi[k]);
            }
          }
        }
      lpart[blk] = lsum;
    }
    free(s);
  }
  double n = (double)H * (double)W;
  csum tot = {0.0, 0.0};
  for (int b = 0; b < nblk; ++b) {
    cs_add(&tot, lpart[b].s);
    cs_add(&tot, lpart[b].c);
  }
  if (grad) {
    double scale = -1.0 / (eps * n);
    for (size_t q = 0; q < NK; ++q) {
      csum t = {0.0, 0.0};
      for (int b = 0; b < nblk; ++b) {
        cs_add(&t, gpart[(size_t)b * NK + q].s);
        cs_add(&t, gpart[(size_t)b * NK + q].c);
      }
      grad[q] = scale * cs_val(&t);
    }
  }
  free(lpart);
  free(gpart);
  return cs_val(&tot) / n;
}

/* eq:Phi and eq:grad with the sum over x restricted to the pixel rows [r0, r1)
   (coordinates of the whole map), unscaled: returns sum_x log p_G(x) and writes
   grad_partial[i*K + k] = sum_x (delta_{i,G(x)} - p_i(x)) psi_k(x) (NULL skips it).
   Summed over a partition of the rows these are n Phi and -(eps n) grad Phi.
   Used for checking row bands of large maps and for timing the oracle on a
   bounded sample. */
double orc_objective_grad_rows(int H, int W, int N, int d, double eps,
                               const double *theta, const int32_t *labels,
                               int r0, int r1, double *grad_partial) {
  int K = orc_num_features(d);
  int A[64], B[64];
  orc_multi_index(d, A, B);
  size_t NK = (size_t)N * K;
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  csum *lp = (csum *)calloc((size_t)nt, sizeof(csum));
  csum *gp = grad_partial ? (csum *)calloc((size_t)nt * NK, sizeof(csum)) : NULL;
#pragma omp parallel
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    double *s = (double *)malloc(sizeof(double) * (size_t)N);
    double psi[64];
#pragma omp for schedule(static)
    for (int r = r0; r < r1; ++r)
      for (int c = 0; c < W; ++c) {
        size_t j = (size_t)r * W + c;
        int g = labels[j];
        pixel_features(r, c, H, W, d, A, B, psi);
        double lse;
        cs_add(&lp[t], pixel_terms(theta, psi, N, K, eps, g, s, &lse));
        if (gp)
          for (int i = 0; i < N; ++i) {
            double w = (i == g ? 1.0 : 0.0) - exp(s[i] - lse);
            for (int k = 0; k < K; ++k) cs_add(&gp[(size_t)t * NK + (size_t)i * K + k], w * psi[k]);
          }
      }
    free(s);
  }
  csum tot = {0.0, 0.0};
  for (int t = 0; t < nt; ++t) cs_add(&tot, cs_val(&lp[t]));
  if (grad_partial)
    for (size_t q = 0; q < NK; ++q) {
      csum a = {0.0, 0.0};
      for (int t = 0; t < nt; ++t) cs_add(&a, cs_val(&gp[(size_t)t * NK + q]));
      grad_partial[q] = cs_val(&a);
    }
  free(lp);
  free(gp);
  return cs_val(&tot);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------
   Unstructured point sets in D = 2 or 3 dimensions (Section 2.1 with Omega any
   finite set of points of [-1,1]^D; Section 3.3's tensor-product basis).
   Multi-indices, degree-graded: for k = 0..d, in 2-D (k - b, b) for b = 0..k
   (the grid's order), in 3-D (k - b - c, b, c) for c = 0..k, then b = 0..k - c. */
int orc_points_num_features(int D, int d) {
  return D == 2 ? (d + 1) * (d + 2) / 2 : (d + 1) * (d + 2) * (d + 3) / 6;
}

static int points_multi_index(int D, int d, int *A, int *B, int *C) {
  int idx = 0;
  for (int k = 0; k <= d; ++k) {
    if (D == 2) {
      for (int b = 0; b <= k; ++b) {
        A[idx] = k - b;
        B[idx] = b;
        C[idx] = 0;
        ++idx;
      }
    } else {
      for (int c = 0; c <= k; ++c)
        for (int b = 0; b <= k - c; ++b) {
          A[idx] = k - b - c;
          B[idx] = b;
          C[idx] = c;
          ++idx;
        }
    }
  }
  return idx;
}

/* psi(x_j) of every point: out[k*n + j] = (P_a(x_j1) P_b(x_j2)) P_c(x_j3)
   (the last factor only in 3-D), the 1-D values from orc_legendre. */
void orc_points_features(int64_t n, int D, int d, const double *X, double *out) {
  int A[256], B[256], C[256];
  int K = points_multi_index(D, d, A, B, C);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    double P[3][16];
    for (int q = 0; q < D; ++q) orc_legendre(X[j * D + q], d, P[q]);
    for (int k = 0; k < K; ++k) {
      double v = P[0][A[k]] * P[1][B[k]];
      if (D == 3) v = v * P[2][C[k]];
      out[(size_t)k * n + j] = v;
    }
  }
}

/* F_theta on a point set (smallest index on ties, -1 on a NaN score) with the
   scores in the canonical order of score(); returns the NaN count and writes
   the number of points with F = G to *n_correct (labels may be NULL). */
int64_t orc_points_assign(int64_t n, int D, int N, int d, const double *theta,
                          const double *X, const int32_t *labels, int32_t *out,
                          int64_t *n_correct) {
  int A[256], B[256], C[256];
  int K = points_multi_index(D, d, A, B, C);
  int64_t correct = 0, nan_count = 0;
#pragma omp parallel for schedule(static) reduction(+ : correct, nan_count)
  for (int64_t j = 0; j < n; ++j) {
    double P[3][16], psi[256];
    for (int q = 0; q < D; ++q) orc_legendre(X[j * D + q], d, P[q]);
    for (int k = 0; k < K; ++k) {
      double v = P[0][A[k]] * P[1][B[k]];
      if (D == 3) v = v * P[2][C[k]];
      psi[k] = v;
    }
    int best = 0;
    double fbest = score(theta, psi, K);
    int bad = isnan(fbest);
    for (int i = 1; i < N; ++i) {
      double f = score(theta + (size_t)i * K, psi, K);
      if (isnan(f)) bad = 1;
      if (f < fbest) {
        fbest = f;
        best = i;
      }
    }
    int lab = bad ? -1 : best;
    if (out) out[j] = lab;
    if (bad) nan_count++;
    if (labels && lab == labels[j]) correct++;
  }
  if (n_correct) *n_correct = correct;
  return nan_count;
}
