/*
 * oracle_driver.c -- runs every function of the CPU oracle (test
 * infrastructure) on small inputs, including its edge cases, so that a build
 * under AddressSanitizer and UndefinedBehaviorSanitizer can check it for
 * out-of-bounds accesses, leaks and undefined arithmetic.  Exits 0 when
 * every call returns the expected status.  CPU only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_num_threads(void);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_gauss_entry(uint64_t seed, uint32_t stream, uint32_t row, uint64_t col, double out[2]);
void orc_gaussian_rowmajor(int64_t rows, int64_t cols, uint64_t seed, uint32_t stream,
                           double *out, int64_t ld);
int64_t orc_srft_row(uint64_t seed, uint64_t i, int64_t m);
double orc_srft_phase(uint64_t seed, uint64_t p);
void orc_srft_operator(int64_t l, int64_t m, uint64_t seed, double *out, int64_t ld);
void orc_sketch(int64_t m, int64_t n, int64_t l, const double *A, int64_t lda,
                const double *G, int64_t ldg, double *Y, int64_t ldy);
void orc_sketch_seeded(int64_t m, int64_t nc, int64_t l, const double *Acols, int64_t lda,
                       uint64_t seed, double *Ycols, int64_t ldy);
int orc_select(int64_t l, int64_t n, int64_t k, const double *Y, int64_t ldy,
               double rank_tol, int64_t *J, double *R, int64_t ldr, double *gaps);
int orc_select_forced(int64_t l, int64_t n, int64_t k, const double *Y, int64_t ldy,
                      double rank_tol, const int64_t *forced, int64_t *J, double *R,
                      int64_t ldr, double *gaps, int64_t *argmax, double *ratio);
int orc_interp(int64_t n, int64_t k, const double *R, int64_t ldr, const int64_t *J,
               double *P, int64_t ldp);
int orc_residual(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                 const int64_t *J, const double *P, int64_t ldp, const double *x0, int q,
                 double *sigma, double *hist);

static int fails = 0;
#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

static double *cmat(int64_t rows, int64_t cols) {
  return (double *)calloc((size_t)(2 * rows * cols), sizeof(double));
}

/* A = X W (rank r) + eps N, column-major m x n, drawn from the oracle's own
 * Gaussian stream (streams 2, 3, 4). */
static double *lowrank(int64_t m, int64_t n, int64_t r, double eps, uint64_t seed) {
  double *A = cmat(m, n);
  double x[2], w[2], e[2];
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < m; ++i) {
      double sr = 0, si = 0;
      for (int64_t t = 0; t < r; ++t) {
        orc_gauss_entry(seed, 2, (uint32_t)i, (uint64_t)t, x);
        orc_gauss_entry(seed, 3, (uint32_t)t, (uint64_t)j, w);
        sr += x[0] * w[0] - x[1] * w[1];
        si += x[0] * w[1] + x[1] * w[0];
      }
      orc_gauss_entry(seed, 4, (uint32_t)i, (uint64_t)j, e);
      A[2 * (i + j * m)] = sr + eps * e[0];
      A[2 * (i + j * m) + 1] = si + eps * e[1];
    }
  return A;
}

static void one_id(int64_t m, int64_t n, int64_t k, int64_t l, double eps, int q, int expect) {
  double *A = lowrank(m, n, k, eps, 7);
  double *G = cmat(l, m), *Y = cmat(l, n), *R = cmat(k, n), *P = cmat(k, n), *x0 = cmat(1, n);
  double *gaps = (double *)calloc((size_t)k, sizeof(double));
  double *hist = (double *)calloc((size_t)q, sizeof(double));
  int64_t *J = (int64_t *)calloc((size_t)k, sizeof(int64_t));
  int64_t *am = (int64_t *)calloc((size_t)k, sizeof(int64_t));
  double *ratio = (double *)calloc((size_t)k, sizeof(double));
  orc_gaussian_rowmajor(l, m, 0, 0, G, m);
  orc_sketch(m, n, l, A, m, G, m, Y, l);
  const int st = orc_select(l, n, k, Y, l, 1e-12, J, R, k, gaps);
  EXPECT(st == expect);
  if (st == 0) {
    EXPECT(orc_select_forced(l, n, k, Y, l, 1e-12, J, J, R, k, gaps, am, ratio) == 0);
    for (int64_t t = 0; t < k; ++t) EXPECT(am[t] == J[t] && ratio[t] == 1.0);
    EXPECT(orc_interp(n, k, R, k, J, P, k) == 0);
    orc_gaussian_rowmajor(1, n, 0, 1, x0, n);
    double sigma = -1.0;
    EXPECT(orc_residual(m, n, k, A, m, J, P, k, x0, q, &sigma, hist) == 0);
    EXPECT(sigma >= 0.0 && isfinite(sigma));
  }
  free(A); free(G); free(Y); free(R); free(P); free(x0); free(gaps); free(hist); free(J);
  free(am); free(ratio);
}

int main(void) {
  uint32_t ctr[4] = {0, 1, 2, 3}, key[2] = {4, 5}, out[4];
  orc_philox4x32_10(ctr, key, out);
  EXPECT(orc_num_threads() >= 1);
  for (uint64_t i = 0; i < 100; ++i) {
    const int64_t s = orc_srft_row(9, i, 37);
    EXPECT(s >= 0 && s < 37);
    const double ph = orc_srft_phase(9, i);
    EXPECT(ph > 0.0 && ph < 1.0);
  }
  {
    double *F = cmat(5, 16);
    orc_srft_operator(5, 16, 3, F, 16);
    free(F);
  }
  one_id(60, 40, 6, 10, 1e-9, 5, 0);     /* an ordinary ID */
  one_id(30, 12, 12, 12, 1e-9, 3, 0);    /* k = n = l: no T */
  one_id(25, 30, 1, 1, 1e-9, 4, 0);      /* k = l = 1 */
  one_id(40, 30, 4, 8, 0.0, 3, 0);       /* exactly rank k */
  {
    /* rank failure: rank-3 input, k = 5 */
    double *A = lowrank(40, 30, 3, 0.0, 8);
    double *G = cmat(8, 40), *Y = cmat(8, 30), *R = cmat(5, 30), *gaps = calloc(5, sizeof(double));
    int64_t J[5], forced[5] = {-1, -1, -1, -1, -1};
    orc_gaussian_rowmajor(8, 40, 0, 0, G, 40);
    orc_sketch(40, 30, 8, A, 40, G, 40, Y, 8);
    EXPECT(orc_select(8, 30, 5, Y, 8, 1e-12, J, R, 5, gaps) == 5);
    EXPECT(orc_select_forced(8, 30, 5, Y, 8, 1e-12, forced, J, R, 5, gaps, NULL, NULL) == 5);
    forced[0] = 30;                                    /* out of range */
    EXPECT(orc_select_forced(8, 30, 5, Y, 8, 1e-12, forced, J, R, 5, gaps, NULL, NULL) == 1);
    free(A); free(G); free(Y); free(R); free(gaps);
  }
  {
    /* argument errors and a zero matrix */
    double *Z = cmat(6, 4), *R = cmat(2, 4), P[16];
    int64_t J[2] = {0, 0};
    EXPECT(orc_select(6, 4, 5, Z, 6, 1e-12, J, R, 5, NULL) == 1);        /* k > n */
    EXPECT(orc_select(6, 4, 2, Z, 6, 1e-12, J, R, 2, NULL) == 5);        /* zero: rank */
    EXPECT(orc_interp(4, 2, R, 2, J, P, 2) == 1);                        /* repeated pivot */
    double sigma, hist[3], x0[8] = {1, 0, 0, 0, 0, 0, 0, 0};
    int64_t J1[1] = {0};
    double P1[8] = {1, 0, 0, 0, 0, 0, 0, 0};
    EXPECT(orc_residual(6, 4, 1, Z, 6, J1, P1, 1, x0, 3, &sigma, hist) == 0);
    EXPECT(sigma == 0.0);
    EXPECT(orc_residual(6, 4, 1, Z, 6, J1, P1, 1, x0, 0, &sigma, hist) == 1);   /* q < 1 */
    free(Z); free(R);
  }
  {
    double *A = lowrank(20, 5, 2, 1e-9, 3), *Ys = cmat(4, 2);
    orc_sketch_seeded(20, 2, 4, A, 20, 11, Ys, 4);
    free(A); free(Ys);
  }
  if (fails) {
    fprintf(stderr, "%d check(s) failed\n", fails);
    return 1;
  }
  printf("oracle under sanitizers: all checks passed\n");
  return 0;
}
