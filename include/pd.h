/*
 * pd.h -- C ABI of the MI355X (gfx950) polynomial-diagram library (libpd.so).
 *
 * Paper: Bourne, Buze, Gallouet, Merigot, "Polynomial diagrams for
 * microstructure modelling" (arXiv 2605.20816).
 *
 * The library fits Legendre polynomial diagrams to labelled pixel grain maps.
 * For a grain map G : Omega -> {0..N-1} on an H x W pixel grid, degree d and
 * eps > 0, with K = (d+1)(d+2)/2 features per grain and parameters
 * theta in R^{N x K}, it evaluates
 *   Phi(theta) = (1/n) sum_x log p_{G(x)}(x),
 *   p_i(x)     = exp(-h_i(x)/eps) / sum_j exp(-h_j(x)/eps),
 *   h_i(x)     = theta_i . psi(x),   psi_(a,b)(x) = P_a(x1) P_b(x2)
 * (Section 2.2 eq. log-res, Section 3.3 eq. h-degree-d-legendre), its gradient
 * (Proposition 4.4, eq. grad), the hard assignment F_theta (Section 2.1) and
 * maximises Phi with L-BFGS (Section 5.2).  The sum form L = n * Phi.
 *
 * Conventions (fixed here where the paper leaves a choice):
 *   - pixel (r, c) has row-major index r*W + c and centre
 *     x1 = (2c + 1 - W)/W, x2 = (2r + 1 - H)/H (Section 2.1, axes rescaled
 *     independently for rectangles, Section 3.3);
 *   - grains and labels are 0-based; ties in F_theta go to the smallest index;
 *   - feature alpha = (a, b) of total degree k sits at index k(k+1)/2 + b
 *     (degree-graded, then b ascending: d = 1 gives 1, x, y);
 *   - theta is N x K row-major FP64 (grain i's K coefficients contiguous).
 *
 * Memory: every pointer is a DEVICE pointer unless marked (host).  The caller
 * owns all buffers; the library never returns memory for the caller to free
 * (other than the context itself).  A context owns its device workspace, which
 * it grows on demand and frees in pd_destroy.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 * pd_features, pd_objective_grad, pd_assign and the warm-start calls are
 * stream-ordered and asynchronous; pd_fit returns when every map has stopped.
 *
 * Errors: arguments that can be checked on the host are checked before any
 * launch (PD_ERR_INVALID_ARG, message in pd_last_error).  HIP failures return
 * PD_ERR_HIP with hipGetErrorString's text.  A context is not thread-safe.
 */
#ifndef PD_H
#define PD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PD_OK = 0,
  PD_ERR_INVALID_ARG = 1,
  PD_ERR_UNSUPPORTED = 2,
  PD_ERR_OOM = 3,
  PD_ERR_HIP = 4,
  PD_ERR_NONFINITE = 5,
  PD_ERR_NOT_CONVERGED = 6
} pd_status;

/* Arithmetic of the logit/exp/gradient contractions.  Global reductions of Phi
 * and grad Phi are FP64 in every mode.
 *   PD_FP64: everything FP64 (the paper's precision, Section 5.1).
 *   PD_FP32: logits, running maxima and log-sum-exp formed in FP64 from FP64 row
 *            coefficients; exponentials and per-row partial sums in FP32; FP64
 *            reductions.
 *   PD_BF16: logit and gradient contractions on the matrix cores, per pixel row
 *            on the row coefficients (three-piece bf16 logit operands, FP16
 *            gradient weights, FP32 accumulation), FP32 log-sum-exp, FP64
 *            reductions; degree <= 6. */
typedef enum { PD_FP64 = 0, PD_FP32 = 1, PD_BF16 = 2 } pd_precision;

/* Gauge of the fit (Lemma 4.2, Remark 4.3).  LAST_ZERO keeps theta_{N-1} = 0
 * (the paper's choice, Section 5.1); CENTERED keeps sum_i theta_i = 0. */
typedef enum { PD_GAUGE_LAST_ZERO = 0, PD_GAUGE_CENTERED = 1, PD_GAUGE_NONE = 2 } pd_gauge;

/* Start of the fit: the caller's theta, theta = 0 (Section 5.2), the learned
 * warm start (network prediction from per-grain descriptors, scaled; see
 * pd_warm_start) or the moment seed of Section 5.6.2, scaled the same way. */
typedef enum { PD_INIT_GIVEN = 0, PD_INIT_ZERO = 1, PD_INIT_MLP = 2, PD_INIT_HEURISTIC = 3 } pd_init;

#define PD_MAX_DEGREE 8

/* One grain map.  labels: DEVICE int32[height*width], values in [0, n_grains)
 * (precondition of the hot calls; pd_validate checks it).  n_grains >= 2
 * (Section 2.1 takes N > 1), 1 <= degree <= PD_MAX_DEGREE, eps > 0 finite. */
typedef struct {
  int32_t height, width;
  const int32_t *labels;
  int32_t n_grains, degree;
  double eps;
} pd_problem;

typedef struct pd_ctx pd_ctx;

/* Create a context on HIP device `device`.  *out receives the handle. */
pd_status pd_create(int device, pd_ctx **out);
/* Free the context and its workspace.  NULL is ignored. */
void pd_destroy(pd_ctx *ctx);
/* Text of the last non-OK status of this context ("" if none). */
const char *pd_last_error(const pd_ctx *ctx);
/* K_d = (d+1)(d+2)/2 (Section 3.1); 0 for d outside [0, PD_MAX_DEGREE]. */
int32_t pd_num_features(int32_t degree);

/* Design matrix eta_L(Omega) of Section 3.3: out[alpha*n + j] = psi_alpha(x_j),
 * n = height*width, alpha in the order above.  out_prec PD_FP64 writes doubles
 * (bit-identical to the canonical recurrence (m+1)P_{m+1} = fma((2m+1)t, P_m,
 * -m P_{m-1}) followed by one correctly rounded division, and one rounded product
 * P_a(x1)*P_b(x2)); PD_FP32 writes floats (the FP64 values rounded); PD_BF16
 * writes two bf16 planes, hi = bf16(psi) then lo = bf16(psi - hi), each K x n. */
pd_status pd_features(pd_ctx *ctx, int32_t height, int32_t width, int32_t degree,
                      pd_precision out_prec, void *out, void *stream);

/* Check that every label of each map lies in [0, n_grains).  Synchronous;
 * returns PD_ERR_INVALID_ARG naming the first bad map. */
pd_status pd_validate(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                      void *stream);

/* Objective Phi (eq. Phi) and gradient (eq. grad) of n_probs maps in one call.
 *   theta    (host array of n_probs DEVICE pointers) N_p x K_p FP64 each;
 *   phi_out  DEVICE double[n_probs]: Phi of each map (mean, <= 0);
 *   grad_out (host array; NULL, or entries NULL, to skip the gradient) DEVICE
 *            N_p x K_p FP64 each: grad Phi, not gauge-projected.
 * Non-finite theta yields NaN outputs.  Labels outside [0, N) yield NaN Phi. */
pd_status pd_objective_grad(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                            const double *const *theta /*host*/, double *phi_out,
                            double *const *grad_out /*host*/, pd_precision prec,
                            void *stream);

/* Allocation-free variant of pd_objective_grad, for callers that cannot
 * allocate device memory during the call (code under stream capture into a
 * graph, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, operation, layouts and results as pd_objective_grad (the same
 * kernels run), but every scratch buffer of the evaluation lives in one fixed
 * device array of PD_NOALLOC_SCRATCH_BYTES bytes per device, set up by
 * pd_create, and nothing is allocated: no hipMalloc, hipFree or pinned host
 * memory, and the plan records are written by a kernel.
 * Limits: at most PD_NOALLOC_MAX_MAPS maps per call (else PD_ERR_INVALID_ARG);
 * an evaluation whose scratch exceeds the array returns PD_ERR_UNSUPPORTED
 * before any launch (roughly: FP32 up to a 1024 x 1024 map with 1000 grains at
 * degree 4; FP64 about half of that).  Every call on one device shares that
 * device's array and leaves its contents there: calls that overlap on one device
 * (other streams, other contexts or host threads) race.  Stream-ordered. */
#define PD_NOALLOC_SCRATCH_BYTES (64u << 20)
#define PD_NOALLOC_MAX_MAPS 4
pd_status pd_objective_grad_noalloc(pd_ctx *ctx, const pd_problem *probs /*host*/,
                                    int32_t n_probs, const double *const *theta /*host*/,
                                    double *phi_out, double *const *grad_out /*host*/,
                                    pd_precision prec, void *stream);

/* Flags of pd_objective_grad_rows. */
/* The form pd_fit evaluates: the indicator moments m_i = sum_{x in G_i} psi(x) of
 * eq. grad are computed once per call (FP64, fixed order) and subtracted from the
 * sums of p_i psi by the FP64 reduction, instead of subtracting psi inside the
 * gradient kernel.  In this form the grains' row coefficients are also kept in
 * the Morton order of their centroids (maps of at most 8192 grains), and the
 * gradient skips the rows of a tile where every term of its 64 grains lies below
 * 2^-96 (FP64) or 2^-48 (FP32) of the pixel's largest, as the objective kernel
 * skips such chunks in every form: a pixel loses at most N 2^-96 (N 2^-48) of its
 * probability mass, below the rounding of its sums.  FP64 / FP32 only (the BF16
 * kernels always apply the one-hot term in place and skip nothing; the flag is
 * accepted and has no effect there). */
#define PD_EVAL_ONEHOT_PRECOMPUTED 1

/* Phi and grad Phi restricted to a band of pixel rows (eq. log-res and eq. grad
 * with the sum over x limited to the rows [rows[2p], rows[2p+1]) of map p):
 *   phi_out[p]  = (1/n) sum_{x in rows} log p_{G(x)}(x),
 *   grad_out[p] = (1/(eps n)) sum_{x in rows} (p(x) - delta_{G(x)}) psi(x),
 * with n = height * width of the whole map, so the bands of a partition of the
 * rows sum to Phi and grad Phi (up to rounding).  This is the share of one device
 * when a map is split by pixel rows (Phi and its gradient are sums over pixels).
 * rows (host, 2 * n_probs int32): 0 <= begin <= end <= height, else
 * PD_ERR_INVALID_ARG; an empty band gives 0 and a zero gradient.  Coordinates
 * and Legendre tables are those of the whole map.  flags: 0 or
 * PD_EVAL_ONEHOT_PRECOMPUTED.  Other arguments, layout and errors as in
 * pd_objective_grad (rows = (0, height) for every map, flags 0, is exactly
 * pd_objective_grad).  Stream-ordered. */
pd_status pd_objective_grad_rows(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                                 const int32_t *rows /*host*/, const double *const *theta /*host*/,
                                 double *phi_out, double *const *grad_out /*host*/,
                                 pd_precision prec, int32_t flags, void *stream);

/* Diagonal of the Hessian of -Phi (eq. hess of Proposition 4.4):
 * diag_out[p][i*K + k] = (1 / (eps^2 n)) sum_x p_i(x) (1 - p_i(x)) psi_k(x)^2 >= 0,
 * the preconditioner of pd_fit.  theta: host array of DEVICE N_p x K_p FP64;
 * diag_out: host array of DEVICE N_p x K_p FP64.  PD_FP64 or PD_FP32 arithmetic
 * (PD_BF16: PD_ERR_UNSUPPORTED).  Stream-ordered. */
pd_status pd_hessian_diag(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                          const double *const *theta /*host*/, double *const *diag_out /*host*/,
                          pd_precision prec, void *stream);

/* Hessian-vector product of -Phi (eq. hess of Proposition 4.4): for each map,
 *   hv_out[p][i*K + k] = (1 / (eps^2 n)) sum_x p_i(x) (u_i(x) - ubar(x)) psi_k(x),
 *   u_i = v_i . psi,  ubar = sum_j p_j u_j,
 * with p the softmax at theta (so v . Hv = (1 / (eps^2 n)) sum_x Var_p(u) >= 0,
 * zero along the gauge direction v_i = c for all i).  The product the Newton-CG
 * solver of pd_fit_newton_cg takes, without forming the NK x NK matrix.
 * theta, v: host arrays of DEVICE N_p x K_p FP64 (Legendre basis); hv_out: host
 * array of DEVICE N_p x K_p FP64, overwritten (it may not alias theta or v).
 * PD_FP64 or PD_FP32 (exponentials and pixel sums in FP32, tile sums in FP64);
 * PD_BF16: PD_ERR_UNSUPPORTED.  Scratch from the context workspace.
 * Stream-ordered. */
pd_status pd_hessian_vec(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                         const double *const *theta /*host*/, const double *const *v /*host*/,
                         double *const *hv_out /*host*/, pd_precision prec, void *stream);

/* ------------------------------------------------------------------------
 * Unstructured point sets in 2-D and 3-D.  Section 2.1 takes the domain as any
 * finite set of points (nothing in the method needs a grid or two dimensions);
 * the basis is Section 3.3's tensor product in D dimensions,
 *   psi_alpha(x) = P_{alpha_1}(x_1) P_{alpha_2}(x_2) [P_{alpha_3}(x_3)], |alpha| <= d,
 * formed as (P_a(x1) P_b(x2)) P_c(x3) from the three-term recurrence with one
 * fused multiply-add per step.  Multi-indices in the degree-graded order: in 2-D
 * (k - b, b) for b = 0..k (the grid's order), in 3-D (k - b - c, b, c) for
 * c = 0..k, then b = 0..k - c; K = (d+1)(d+2)/2 or (d+1)(d+2)(d+3)/6.
 * Without a grid the logit costs K FMAs per (point, grain). */
#define PD_POINTS_DMAX2 7
#define PD_POINTS_DMAX3 4
#define PD_POINTS_KMAX 36
typedef struct {
  const double *coords;   /* DEVICE n_points x dim FP64, row-major, in [-1, 1]^dim */
  const int32_t *labels;  /* DEVICE n_points, values in [0, n_grains)             */
  int64_t n_points;       /* >= 1                                                 */
  int32_t dim;            /* 2 or 3                                               */
  int32_t n_grains;       /* >= 2                                                 */
  int32_t degree;         /* 2-D: 0..PD_POINTS_DMAX2; 3-D: 0..PD_POINTS_DMAX3     */
  double eps;             /* > 0                                                  */
} pd_points;

/* K of a point set of this dimension and degree (0 for an invalid dimension). */
int32_t pd_points_num_features(int32_t dim, int32_t degree);

/* Phi (eq. log-res) and grad Phi (eq. grad) of each point set, the definitions of
 * pd_objective_grad with the sum over the points: phi_out DEVICE double[n_probs];
 * grad_out host array of DEVICE N x K FP64 (the array or an entry may be NULL:
 * Phi only); theta host array of DEVICE N x K FP64.  PD_FP64 (everything FP64) or
 * PD_FP32 (logits and log-sum-exp FP64, exponentials and per-point sums FP32);
 * PD_BF16: PD_ERR_UNSUPPORTED.  A grain whose logit lies 96 (FP64) or 48 (FP32)
 * base-2 units below the running maximum of every point of a 64-point wave is
 * left out of that wave's sums (at most N 2^-96 / N 2^-48 of a point's mass).
 * Labels are a precondition (not checked).  Scratch from the context workspace
 * (n K + 3 n + chunks N_pad K doubles).  Stream-ordered. */
pd_status pd_points_objective_grad(pd_ctx *ctx, const pd_points *probs /*host*/, int32_t n_probs,
                                   const double *const *theta /*host*/, double *phi_out,
                                   double *const *grad_out /*host*/, pd_precision prec,
                                   void *stream);

/* F_theta of each point set (Section 2.1, smallest index on ties, -1 where a
 * score is NaN) with the scores theta_i0 then one FMA per feature in index
 * order, in FP64: labels_out host array of DEVICE int32[n_points] (the array or
 * an entry may be NULL); n_correct_out DEVICE int64[n_probs]: #{x : F(x) = G(x)}.
 * Stream-ordered. */
pd_status pd_points_assign(pd_ctx *ctx, const pd_points *probs /*host*/, int32_t n_probs,
                           const double *const *theta /*host*/, int32_t *const *labels_out /*host*/,
                           int64_t *n_correct_out, void *stream);

/* Hard assignment F_theta (Section 2.1, smallest index on ties) in FP64 with the
 * canonical score order f = theta_i0, f = fma(theta_ik, psi_k, f), k = 1..K-1,
 * so labels are bit-reproducible.  labels_out (host array; entries may be NULL)
 * DEVICE int32[n] each (-1 where a score is NaN); n_correct_out DEVICE
 * int64[n_probs]: #{x : F(x) = G(x)} (Acc = n_correct / n, Section 2.2). */
pd_status pd_assign(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                    const double *const *theta /*host*/, int32_t *const *labels_out /*host*/,
                    int64_t *n_correct_out, void *stream);

/* ------------------------------------------------------------------------
 * Warm start.  Per grain i (pixels G_i, n pixels, N grains):
 *   frame   (PD_FRAME_DIM doubles): centroid y'_i (eq. centroid-guess), radius
 *           r_i = 2 sqrt(lambda_max(B'_i)) (at least one pixel width
 *           2 / max(H, W)), central second moments B11, B12, B22 (eq. cov-guess,
 *           in x units), pixel count |G_i|, 0.  Empty grains: (0, 0, 1, 0, ...).
 *   descriptor (PD_DESC_DIM floats): log(N |G_i| / n); the 27 Legendre indicator
 *           moments mean over G_i of P_a(x_1) P_b(x_2), 1 <= a + b <= 6, in the
 *           degree-graded order; N B11, N B12, N B22; log(N) / 10.  Zero for
 *           empty grains.  Exact integer pixel sums and a fixed summation order
 *           make them bitwise reproducible.
 *   moment seed theta'_i (Section 5.6.2): A'_i = B'_i^{-1} (eq. A-guess; the
 *           identity at degree 1), w'_i = sqrt(det A'_i) area(G_i) / pi, the
 *           ratio of the grain's area (4 |G_i| / n on [-1, 1]^2) to the area of
 *           the ellipse of B'_i (eq. w-guess and the sentence after it), the score
 *           (x - y')^T A' (x - y') - w' of eq. h-APD in the Legendre basis
 *           (x^2 = (2 P_2(x) + 1) / 3); at degree 1 the common |x|^2 is dropped (a
 *           gauge term, Lemma 4.2); coefficients of degree >= 3 are zero.
 *   Empty grains get the row (C, 0, ..., 0), C = 1 + max_i sum_k |theta_ik|, a
 *           score above every other grain's on [-1, 1]^2, so they win no pixel.
 * The network maps a descriptor to theta_i in the global Legendre basis, in the
 * normalisation of pd_warm_targets (K_d outputs). */
#define PD_DESC_DIM 32
#define PD_FRAME_DIM 8
#define PD_MLP_IN PD_DESC_DIM
#define PD_MLP_WIDTH 256

/* Networks by degree: params[d] is a DEVICE FP32 buffer of pd_mlp_num_params(K_d)
 * floats for maps of degree d, or NULL (those maps use the moment seed alone). */
typedef struct pd_mlp {
  const float *params[PD_MAX_DEGREE + 1];
} pd_mlp;

/* Parameter count of the network 32 -> 256 -> 256 -> k_out with GELU
 * (0.5 z (1 + erf(z / sqrt 2))) after both hidden layers.  Buffer layout:
 * W1 (32 x 256, input-major), b1 (256), W2 (256 x 256), b2, W3 (256 x k_out), b3;
 * layer l computes z = x W_l + b_l.  0 if k_out < 1. */
int64_t pd_mlp_num_params(int32_t k_out);

/* Descriptors and frames of every grain of each map.  desc_out: host array of
 * DEVICE float[N_p x PD_DESC_DIM]; frame_out: host array (NULL, or NULL entries,
 * to skip) of DEVICE double[N_p x PD_FRAME_DIM].  Stream-ordered.  Labels must
 * lie in [0, N) (pixels with other labels are ignored). */
pd_status pd_descriptors(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                         float *const *desc_out /*host*/, double *const *frame_out /*host*/,
                         void *stream);

/* Moment seed theta' (unscaled) of each map: theta_out host array of DEVICE
 * N_p x K_p FP64.  Stream-ordered. */
pd_status pd_heuristic(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                       double *const *theta_out /*host*/, void *stream);

/* Training targets from fitted parameters: theta_fit centred over the non-empty
 * grains (a common shift is a gauge, Lemma 4.2) and divided by its root mean
 * square over those grains and the K coefficients (the scale of a fit is free,
 * Proposition 4.8); zero rows for empty grains.  theta_fit: host array of DEVICE
 * N_p x K_p FP64; target_out: host array of DEVICE float[N_p x K_p]; lambda_out:
 * DEVICE double[n_probs] (the RMS) or NULL.  Stream-ordered. */
pd_status pd_warm_targets(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                          const double *const *theta_fit /*host*/,
                          float *const *target_out /*host*/, double *lambda_out,
                          void *stream);

/* Network forward pass on `batch` rows of x (DEVICE float[batch x PD_MLP_IN]) into
 * y_out (DEVICE float[batch x k_out]).  PD_FP32: FP32 arithmetic (the training
 * forward pass); PD_BF16: weights and activations rounded to bf16 on the matrix
 * cores, FP32 accumulation and bias.  Stream-ordered. */
pd_status pd_mlp_forward(pd_ctx *ctx, int32_t k_out, const float *params, const float *x,
                         int32_t batch, pd_precision prec, float *y_out, void *stream);

/* Loss mean((y - target)^2) over batch x k_out outputs of the FP32 forward pass
 * (loss_out: DEVICE double[1]) and its gradient with respect to every parameter
 * (grad_out: DEVICE float[pd_mlp_num_params(k_out)], same layout as params).
 * Deterministic (fixed summation order).  Stream-ordered. */
pd_status pd_mlp_backward(pd_ctx *ctx, int32_t k_out, const float *params, const float *x,
                          const float *target, int32_t batch, double *loss_out, float *grad_out,
                          void *stream);

/* One Adam step (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps); step >= 1.
 * All arrays DEVICE float[n_params].  Stream-ordered. */
pd_status pd_mlp_adam(pd_ctx *ctx, int64_t n_params, float *params, const float *grad, float *m,
                      float *v, int32_t step, float lr, float beta1, float beta2, float eps,
                      void *stream);

/* Warm start of each map: theta_hat = the network outputs for the map's grains
 * (BF16 inference), centred over its non-empty grains, or the moment seed where
 * mlp or mlp->params[d] is NULL; empty grains get the row that wins no pixel.
 * Then theta = s* theta_hat with s* maximising the concave restriction
 * s -> Phi(s theta_hat) (Proposition 4.4): bracketing in log2 s by steps of 2
 * from s0 = eps max(H, W) / (28 sqrt N) (at most 12 steps), then 6 golden-section
 * evaluations; the best evaluated point is kept.  If Phi(s* theta_hat) < Phi(0)
 * = -log N the map falls back to theta = 0.  The search evaluates Phi in FP64 for
 * prec PD_FP64, in FP32 otherwise.  theta_out: host array of DEVICE N_p x K_p
 * FP64; scale_out (host, may be NULL): s* per map (0 after a fall-back).
 * Synchronous. */
pd_status pd_warm_start(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                        const pd_mlp *mlp /*host, may be NULL*/, double *const *theta_out /*host*/,
                        pd_precision prec, double *scale_out /*host*/, void *stream);

/* L-BFGS fit (Section 5.2) of n_probs maps at once, on the device.
 * Minimises -Phi with memory `history`, strong-Wolfe line search (c1 = 1e-4,
 * c2 = 0.9, cubic zoom, <= 20 evaluations per search), first trial step
 * 1/||g||_2 when the memory is empty and 1 otherwise; stops a map at the first
 * accepted iterate with FP64 accuracy >= target_acc, at max_iter iterations, or
 * when ||g||_inf <= gtol.  Accuracy is checked every check_every iterations. */
typedef struct {
  pd_precision prec;      /* arithmetic of the objective/gradient evaluations   */
  pd_gauge gauge;         /* PD_GAUGE_LAST_ZERO (paper) or PD_GAUGE_CENTERED     */
  pd_init init;           /* PD_INIT_GIVEN uses theta_inout as the start         */
  int32_t history;        /* L-BFGS memory, 1..32 (default 10)                   */
  int32_t max_iter;       /* iteration budget (paper: 1000 or 2000)              */
  double target_acc;      /* stop at Acc >= target_acc (e.g. 0.99); > 1 disables */
  double gtol;            /* stop at ||grad||_inf <= gtol (0 disables)           */
  int32_t check_every;    /* accuracy / stop-flag poll period in iterations      */
  const struct pd_mlp *mlp; /* PD_INIT_MLP: the networks (see pd_warm_start)    */
  int32_t precondition;   /* 0: H0 = gamma I.  T > 0: H0 = gamma Dinv with
                             Dinv = diag(1 / (D + 1e-6 max D)), D the Hessian
                             diagonal of pd_hessian_diag taken at the start and at
                             every T-th accepted iterate, gamma = s.y / y.Dinv y of
                             the newest pair, every search starting at t = 1.
                             Gauge PD_GAUGE_LAST_ZERO.  With PD_BF16, D comes
                             from an FP32 evaluation at the refresh iterates.      */
  /* Schedule of eps (annealing; Section 5.2 and the end of Section 5.6.4 leave it
   * to future work).  anneal_levels S = 0: one fit at each map's eps.  S > 0:
   * levels eps_k = eps * anneal_factor^(S - k), k = 0 .. S, each an L-BFGS fit
   * (fresh memory) from the previous level's theta; level k < S has a budget of
   * min(anneal_iters, max_iter - k anneal_iters) iterations, the last level
   * max_iter - S anneal_iters.  Since F_theta does not depend on eps (Lemma 4.1),
   * a map stops at the first accepted iterate of any level whose accuracy
   * reaches target_acc.  The report sums iterations, evaluations and times over
   * the levels, gives the status of the map's last level (budget for a map that
   * ran out inside the schedule), and phi = Phi at the map's own eps.  The init
   * modes apply to the first level (the warm start's scale search at eps_0).  */
  int32_t anneal_levels;  /* 0 .. 30                                             */
  double anneal_factor;   /* > 1 when anneal_levels > 0                          */
  int32_t anneal_iters;   /* >= 1 when anneal_levels > 0                         */
  /* Per-iteration metrics (may be NULL): host array of n_probs DEVICE buffers of
   * trace_cap x PD_TRACE_FIELDS doubles (an entry may be NULL).  The k-th accepted
   * iterate of a map (k = 1, 2, ..., counted over all levels of an eps schedule)
   * is written to row (k - 1) % trace_cap of its buffer by the device when it is
   * accepted: a ring that keeps the last trace_cap iterates, read after the call
   * (rows of iterates that were not reached are left as they were). */
  double *const *trace;
  int32_t trace_cap;      /* >= 1 when trace is not NULL                        */
  /* L-BFGS state (may be NULL): host array of n_probs DEVICE buffers of
   * pd_fit_state_size(N_p, degree_p, history) doubles.  On return each map's
   * state is written there: a header of PD_FIT_STATE_HEADER doubles (format tag,
   * N, K, history, pairs held, ring head, accepted iterations so far, gamma,
   * preconditioner period, gauge), then the ring of history + 1 slots of s and y
   * (N K each), rho, the Gram matrices s_j.y_k and y_j.y_k ((history + 1)^2 each,
   * the latter in the D^-1 metric with the preconditioner) and D^-1 (N K; only
   * meaningful with precondition > 0).  With resume = 1 the fit starts from that
   * state instead of an empty memory: theta_inout must hold the iterate it was
   * written with (PD_INIT_GIVEN), history, gauge, precondition and the map's N
   * and degree must match the header (else PD_ERR_INVALID_ARG), and the
   * iteration count continues from the header's (max_iter counts the iterations
   * of this call; check_every, the preconditioner refreshes and the trace
   * numbering follow the total).  At a resume the Gram matrices of the stored
   * pairs (and, with the preconditioner, gamma and a refresh due at that iterate)
   * are formed again, since a fit that stops at its budget skips them for its
   * last pair, and the first direction comes from the two-loop recursion over the
   * stored pairs; the uninterrupted fit forms it in the compact form, so a
   * resumed trajectory equals the uninterrupted one to rounding, not bit for
   * bit.  Not combined with an eps schedule. */
  double *const *state;
  int32_t resume;         /* 0 or 1                                             */
} pd_fit_opts;

#define PD_FIT_STATE_HEADER 16
/* Doubles of one map's L-BFGS state buffer (pd_fit_opts.state); 0 for invalid
 * arguments (n_grains < 2, degree outside 1..PD_MAX_DEGREE, history outside
 * 1..32).  Host only. */
int64_t pd_fit_state_size(int32_t n_grains, int32_t degree, int32_t history);

/* Fields of one trace row: the iteration k, the objective+gradient evaluations
 * of this call so far (over all levels), Phi at the iterate (at the level's eps under a schedule), the largest
 * |entry| of the gradient at the iterate (in the fit's gauge), the accepted step
 * length t of the line search, and the FP64 accuracy of the iterate (NaN with
 * PD_BF16, whose accuracy is assigned one step later and only at check
 * iterates). */
#define PD_TRACE_FIELDS 6

typedef struct {
  int32_t status;         /* 0 target reached, 1 budget, 2 gtol, 3 line search failed,
                             4 non-finite                                          */
  int32_t iters, evals;   /* accepted iterations, objective+gradient evaluations  */
  double phi, acc;        /* final Phi and accuracy                               */
  double seconds_total;   /* wall time of this pd_fit call                        */
  double seconds_to_target; /* wall time until Acc >= target_acc (-1 if never)    */
  double seconds_iterating; /* device time from the first evaluation's decision to
                               the last accepted iterate: the `iters` iterations,
                               with their evals_iterating evaluations, accuracy
                               checks and L-BFGS updates, without set-up          */
  int32_t evals_iterating;  /* evaluations in that window                          */
} pd_fit_report;

/* theta_inout: host array of DEVICE N_p x K_p FP64 pointers (start if
 * PD_INIT_GIVEN; result on return).  reports: host array of n_probs.
 * PD_INIT_MLP / PD_INIT_HEURISTIC run pd_warm_start first (its time counts in
 * seconds_to_target).  Maps with N K >= 1024 run the long vector passes of an
 * accepted step on several blocks; the environment variable PD_FIT_SPLIT_MIN
 * (read at each call) lowers that size (values above 1024 act as 1024).  A
 * map's result does not depend on the other maps of its batch. */
pd_status pd_fit(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                 double *const *theta_inout /*host*/, const pd_fit_opts *opts /*host*/,
                 pd_fit_report *reports /*host*/, void *stream);

/* Inexact Newton ascent of Phi (Newton-CG) with Hessian-vector products from
 * eq. hess of Proposition 4.4, in the gauge theta_N = 0 (on which the Hessian
 * of -Phi is positive definite, Proposition 4.11).  Per iteration: g = grad(-Phi)
 * with the last grain's row zeroed; conjugate gradients on H d = -g from d = 0
 * (H v by the kernels of pd_hessian_vec, last row zeroed), stopped after cg_max
 * steps, when ||r|| <= min(0.5, sqrt(||g||)) ||g|| (forcing term of Eisenstat
 * and Walker), or at non-positive curvature (d = -g if at the first step); then
 * step halving from t = 1 until -Phi(x + t d) <= -Phi(x) + 1e-4 t g.d.  A map
 * stops at the first iterate (the start included) whose FP64 accuracy (from the
 * certified arg-max of each evaluation) reaches target_acc, when ||g||_inf <=
 * gtol, at max_iter iterations, or when max_halvings halvings fail.  Maps of a
 * batch iterate independently (a stopped map's kernels are gated off).
 * theta_inout: host array of DEVICE N_p x K_p FP64, the start (moved into the
 * gauge) and the result.  Allocates its state (7 N K doubles per map) per call;
 * synchronous (returns after the last phase on `stream`). */
typedef struct {
  pd_precision prec;      /* PD_FP64 or PD_FP32: objective and products        */
  int32_t max_iter;       /* Newton iterations (>= 0)                           */
  int32_t cg_max;         /* CG steps per iteration, 1 .. 10000                 */
  int32_t max_halvings;   /* evaluations per line search, 1 .. 60               */
  double target_acc;      /* stop at Acc >= target_acc; > 1 disables            */
  double gtol;            /* stop at ||grad||_inf <= gtol (0: only at 0)        */
} pd_newton_opts;

typedef struct {
  int32_t status;         /* 0 target, 1 budget, 2 gtol, 3 line search failed,
                             4 non-finite                                       */
  int32_t iters, evals, hvps; /* accepted iterations, objective evaluations,
                             Hessian-vector products                           */
  double phi, acc;        /* Phi and accuracy at the result                     */
  double seconds_total;   /* wall time of the call                              */
  double seconds_to_target; /* wall time until Acc >= target_acc (-1 if never)  */
} pd_newton_report;

pd_status pd_fit_newton_cg(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                           double *const *theta_inout /*host*/, const pd_newton_opts *opts,
                           pd_newton_report *reports /*host*/, void *stream);

/* Physical parameters of a fitted degree-1 (power) or degree-2 (anisotropic
 * power) diagram, Section 5.6.3 with eq. pd-lr-to-phys / apd-lr-to-phys of
 * Section 2.3.1.  The Legendre coefficients (P_2(t) = (3t^2 - 1)/2) are rewritten
 * as h_i(x) = x.A_i x + c_i.x + c_i0, and y_i = -(1/2) A_i^{-1} c_i,
 * w_i = y_i.A_i y_i - c_i0.  The gauge freedom of Lemma 4.2 (adding
 * lambda (x1^2 + x2^2) to every grain changes no cell) is used to make every
 * anisotropy positive definite: lambda = max(0, margin - min_i lambda_min(A_i))
 * and A_i + lambda I is returned.  Degree 1: A_i = I (the common |x|^2 is the
 * gauge term the coefficients already drop), lambda = 0.
 *   theta:      DEVICE n_grains x K FP64 (K = 3 or 6; any gauge);
 *   params_out: DEVICE n_grains x PD_PHYS_DIM FP64, per grain
 *               y1, y2, w, A11, A12, A22;
 *   lambda_out: DEVICE double[1], the shift applied.
 * margin > 0 finite.  Degree outside {1, 2}: PD_ERR_UNSUPPORTED.  Stream-ordered. */
#define PD_PHYS_DIM 6
pd_status pd_recover_params(pd_ctx *ctx, int32_t n_grains, int32_t degree, const double *theta,
                            double margin, double *params_out, double *lambda_out, void *stream);

/* Per-stage timing of one evaluation (the library's tracing hook; not part of
 * the paper).  Runs the evaluation of pd_objective_grad stage by stage, each
 * stage `reps` times back to back between HIP events on `stream`, and writes the
 * average milliseconds per launch of each stage to ms_out (host, PD_NUM_STAGES
 * entries, in the order of pd_stage).  Gradient stages are included.  Synchronous.
 * PD_BF16 times its matrix-core stages in the PD_STAGE_LSE / PD_STAGE_GRAD slots. */
typedef enum {
  PD_STAGE_TABLES = 0,  /* 1-D Legendre tables (and the one-hot term's moments) */
  PD_STAGE_CENTER = 1,  /* grain-mean removal and eps scaling of theta          */
  PD_STAGE_PREP = 2,    /* row coefficients C[r][i][a]                          */
  PD_STAGE_LSE = 3,     /* per-pixel log-sum-exp and partial sums of log p_G,
                           with the certified arg-max (the kernel pd_fit runs)  */
  PD_STAGE_GRAD = 4,    /* partial sums of p psi (the one-hot term precomputed,
                           as in pd_fit)                                        */
  PD_STAGE_REDUCE = 5,  /* fixed-order reductions to Phi and grad Phi           */
  PD_NUM_STAGES = 6
} pd_stage;

pd_status pd_profile_eval(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                          const double *const *theta /*host*/, pd_precision prec, int32_t reps,
                          double *ms_out /*host*/, void *stream);

/* Autotuner of the work decomposition (tile shapes of the gradient kernels:
 * pixel-tile size per 64-grain wave on the FP64/FP32 path, pixel-chunk length
 * per grain group on the BF16 path).  Times one evaluation of the given batch
 * for each candidate (waves per map: 1024 .. 65536; five evaluations each),
 * keeps the fastest for the batch's key (precision, largest degree, log2 of the
 * pixel-grain pairs, number of maps) in the context -- the untuned default
 * (about 2^18 pixel-grain pairs per wave, 8192 to 65536 waves) unless
 * another is more than 2% faster, so that timing noise does not change the
 * tiling, and with it the rounding of the gradient sums, between runs -- and
 * uses it in every later plan with that key.  If
 * the environment variable PD_AUTOTUNE_CACHE names a file, results are read
 * from and appended to it (one "prec dmax size_log2 n_maps waves" line each).
 * Synchronous.  best_waves_out (host, may be NULL) receives the choice. */
pd_status pd_autotune(pd_ctx *ctx, const pd_problem *probs /*host*/, int32_t n_probs,
                      const double *const *theta /*host*/, pd_precision prec,
                      int32_t *best_waves_out /*host*/, void *stream);

/* Microbenchmark of one unit that bounds the evaluation kernels (measurement
 * support; not part of the method).  kind: 0 = FP32 FMA (not packed), 1 = the
 * hardware base-2 exponential v_exp_f32, 2 = four FP32 FMAs per exponential
 * (shows whether the two overlap), 3 = FP64 FMA, 4 = BF16 matrix-core product
 * v_mfma_f32_32x32x16_bf16.  rate_out (host): flop/s for kinds 0, 3 and 4 (two
 * flops per multiply-add), exponentials/s for kinds 1 and 2.  Independent
 * dependency chains in every thread and a full grid, best of five launches
 * timed with HIP events.  Uses the evaluation workspace; synchronous.
 * PD_ERR_INVALID_ARG for another kind. */
pd_status pd_probe_peak(pd_ctx *ctx, int32_t kind, double *rate_out /*host*/, void *stream);

/* The elementary functions of the evaluation kernels on given arguments (a check
 * of their accuracy): out[j] = f(in[j]) for fn 0: the FP64 2^x (arguments <= 0,
 * as the kernels form them), 1: the FP32 2^x of (float)x, 2: the FP64 log2,
 * 3: the FP32 log2 of (float)x; FP32 results widened to FP64.  in, out: DEVICE
 * double[n].  Stream-ordered. */
pd_status pd_probe_math(pd_ctx *ctx, int32_t fn, const double *in, double *out, int64_t n,
                        void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PD_H */
