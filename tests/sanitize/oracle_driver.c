/* Driver of the C oracle for the host AddressSanitizer / UndefinedBehavior-
 * Sanitizer build (test infrastructure; tests/test_oracle_sanitized.py builds
 * and runs it).  Reads a small problem from the binary file named by argv[1],
 * calls every exported oracle function on it, and writes the results to
 * argv[2], so the test can compare them bit for bit with the ordinary build.
 *
 * Input (native endianness): int32 H, W, N, d, D, n_pts; double eps;
 * double theta[N*K]; int32 labels[H*W]; double X[n_pts*D]; double theta_p[N*Kp];
 * int32 labels_p[n_pts]  (K = grid features of d, Kp = point-set features of
 * degree d in D dimensions). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_num_features(int d);
void orc_multi_index(int d, int *a_out, int *b_out);
double orc_coord(int idx, int len);
void orc_legendre(double t, int d, double *P);
void orc_features(int H, int W, int d, double *out);
int64_t orc_assign_rows(int H, int W, int N, int d, const double *theta, const int32_t *labels,
                        int r0, int r1, int32_t *out, int64_t *n_correct);
int64_t orc_assign(int H, int W, int N, int d, const double *theta, const int32_t *labels,
                   int32_t *out, int64_t *n_correct);
double orc_objective_grad(int H, int W, int N, int d, double eps, const double *theta,
                          const int32_t *labels, double *grad);
double orc_objective_grad_rows(int H, int W, int N, int d, double eps, const double *theta,
                               const int32_t *labels, int r0, int r1, double *grad_partial);
int orc_points_num_features(int D, int d);
void orc_points_features(int64_t n, int D, int d, const double *X, double *out);
int64_t orc_points_assign(int64_t n, int D, int N, int d, const double *theta, const double *X,
                          const int32_t *labels, int32_t *out, int64_t *n_correct);

static void *take(FILE *f, size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

static void put(FILE *f, const void *p, size_t bytes) {
  if (fwrite(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short output\n");
    exit(3);
  }
}

int main(int argc, char **argv) {
  if (argc != 3) return 1;
  FILE *in = fopen(argv[1], "rb");
  if (!in) return 1;
  int32_t *hd = (int32_t *)take(in, 6 * sizeof(int32_t));
  const int H = hd[0], W = hd[1], N = hd[2], d = hd[3], D = hd[4], np_ = hd[5];
  double *eps = (double *)take(in, sizeof(double));
  const int K = orc_num_features(d), Kp = orc_points_num_features(D, d);
  const size_t n = (size_t)H * W;
  double *theta = (double *)take(in, sizeof(double) * (size_t)N * K);
  int32_t *labels = (int32_t *)take(in, sizeof(int32_t) * n);
  double *X = (double *)take(in, sizeof(double) * (size_t)np_ * D);
  double *theta_p = (double *)take(in, sizeof(double) * (size_t)N * Kp);
  int32_t *labels_p = (int32_t *)take(in, sizeof(int32_t) * (size_t)np_);
  fclose(in);

  FILE *out = fopen(argv[2], "wb");
  if (!out) return 1;
  int a[64], b[64];
  orc_multi_index(d, a, b);
  put(out, a, sizeof(int) * K);
  put(out, b, sizeof(int) * K);
  double c = orc_coord(3, W);
  put(out, &c, sizeof c);
  double P[16];
  orc_legendre(-0.3, d, P);
  put(out, P, sizeof(double) * (d + 1));
  double *feat = (double *)malloc(sizeof(double) * (size_t)K * n);
  orc_features(H, W, d, feat);
  put(out, feat, sizeof(double) * (size_t)K * n);
  double *grad = (double *)malloc(sizeof(double) * (size_t)N * K);
  double phi = orc_objective_grad(H, W, N, d, *eps, theta, labels, grad);
  put(out, &phi, sizeof phi);
  put(out, grad, sizeof(double) * (size_t)N * K);
  /* a band inside the map (the whole map when it has fewer than 3 rows) */
  const int b0 = H > 2 ? 1 : 0, b1 = H > 2 ? H - 1 : H, a0 = H > 2 ? 2 : 0;
  double v = orc_objective_grad_rows(H, W, N, d, *eps, theta, labels, b0, b1, grad);
  put(out, &v, sizeof v);
  put(out, grad, sizeof(double) * (size_t)N * K);
  int32_t *F = (int32_t *)malloc(sizeof(int32_t) * n);
  int64_t nc = 0, nn = orc_assign(H, W, N, d, theta, labels, F, &nc);
  put(out, F, sizeof(int32_t) * n);
  put(out, &nc, sizeof nc);
  put(out, &nn, sizeof nn);
  nn = orc_assign_rows(H, W, N, d, theta, labels, a0, H, F, &nc);
  put(out, F, sizeof(int32_t) * (size_t)(H - a0) * W);
  put(out, &nc, sizeof nc);
  double *fp = (double *)malloc(sizeof(double) * (size_t)Kp * np_);
  orc_points_features(np_, D, d, X, fp);
  put(out, fp, sizeof(double) * (size_t)Kp * np_);
  int32_t *Fp = (int32_t *)malloc(sizeof(int32_t) * (size_t)np_);
  nn = orc_points_assign(np_, D, N, d, theta_p, X, labels_p, Fp, &nc);
  put(out, Fp, sizeof(int32_t) * (size_t)np_);
  put(out, &nc, sizeof nc);
  fclose(out);
  free(hd); free(eps); free(theta); free(labels); free(X); free(theta_p); free(labels_p);
  free(feat); free(grad); free(F); free(fp); free(Fp);
  return 0;
}
