/*
 * rid_oracle.c -- reference CPU implementation of the randomized interpolative
 * decomposition (ID) of a complex matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * Source: Lucas, Stalzer & Feo, "Parallel implementation of fast randomized
 * algorithms for the decomposition of low rank matrices" (arXiv 1205.3830).
 *   Sec. 2, problem statement      : A (m x n, approximate rank k) ~= B P,
 *                                     B = k columns of A, P = [I T].
 *   Sec. 2, randomization          : Y = (random l x m operator) A, l >= k.
 *                                     The paper's operator is S F D; it also
 *                                     allows any faster randomization.  Here
 *                                     the operator is a complex Gaussian G.
 *   Sec. 2, approximate QR         : Y ~= Q R, R = [R1 R2], R1 k x k upper
 *                                     triangular, after a column permutation
 *                                     that brings the k most weighted,
 *                                     independent columns to the front.
 *   Sec. 2, interpolation matrix   : solve R2 = R1 T, then P = [I T].
 *   Sec. 2, failure mode           : rank(Y) < k -> redraw the randomness.
 *   Sec. 3.2, QR method            : classical Gram-Schmidt with a second
 *                                     orthogonalisation pass (CGS2).
 *   Table 5                        : the quantity ||A - B P||_2.
 *
 * Everything is plain loops in IEEE double (complex stored as interleaved
 * re,im pairs, column-major with a leading dimension), except the power
 * iteration for ||A - B P||_2, which runs in binary128 (__float128) because
 * A - B P is ~1e-10 of A and plain double sums lose most of its digits.
 * Compile with -ffp-contract=off so that no FMA changes the double rounding.
 *
 * Parity status of each function is recorded in its comment; every function
 * here is pinned by a CPU test except where a comment says otherwise.
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_RANK 5

/* Threads the OpenMP loops of the oracle use. */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds of the 4x32 Philox S-box with the    */
/* published multipliers and Weyl key increments.  Pinned by the published    */
/* known-answer vectors.                                                      */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n1 = lo1;
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  uint32_t n3 = lo0;
  c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof(c));
}

/* One complex Gaussian draw, Re and Im each N(0, 1/2), E|g|^2 = 1.
 * Counter = (col low word, col high word, row, stream), key = (seed low, seed
 * high).  Two 52-bit uniforms in (0,1) come from the word pairs (w0,w1) and
 * (w2,w3): u = (2x+1) 2^-53 with x the top 52 bits of the 64-bit pair.  The
 * Box-Muller transform in polar form gives g = sqrt(-ln u1) exp(2 pi i u2).
 * The randomness is the method's own draw (Sec. 2 randomization step); its
 * bit pattern is this project's convention, which the GPU library implements
 * separately.                                                                */
static const double ORC_TWO_PI = 6.283185307179586476925286766559;

static double u52(uint32_t lo, uint32_t hi) {
  const uint64_t x = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 12;
  return (double)(2 * x + 1) * 0x1p-53;
}

void orc_gauss_entry(uint64_t seed, uint32_t stream, uint32_t row, uint64_t col,
                     double out[2]) {
  const uint32_t ctr[4] = {(uint32_t)col, (uint32_t)(col >> 32), row, stream};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  const double u1 = u52(w[0], w[1]);
  const double u2 = u52(w[2], w[3]);
  const double rad = sqrt(-log(u1));
  const double ang = ORC_TWO_PI * u2;
  out[0] = rad * cos(ang);
  out[1] = rad * sin(ang);
}

/* rows x cols Gaussian matrix, entry (i, j) drawn with row = i, col = j,
 * written row-major: out[2*(i*ld + j) + {0,1}].                              */
void orc_gaussian_rowmajor(int64_t rows, int64_t cols, uint64_t seed, uint32_t stream,
                           double *out, int64_t ld) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < rows; ++i)
    for (int64_t j = 0; j < cols; ++j)
      orc_gauss_entry(seed, stream, (uint32_t)i, (uint64_t)j, out + 2 * (i * ld + j));
}

/* ------------------------------------------------------------------------ */
/* The paper's own randomization, Y = S F D A (Sec. 2, eqs. (4)-(7)):        */
/*   D = diag(exp(2 pi i phi_p)), phi_p uniform on (0,1)    (stream 5)        */
/*   F(s, p) = exp(-2 pi i s p / m), the unnormalised DFT                    */
/*   S keeps rows s_0..s_{l-1} of F D A, i.i.d. uniform on {0..m-1}, drawn    */
/*     with replacement                                      (stream 6)        */
/* so Y = G A with G(i, p) = exp(2 pi i (phi_p - (s_i p mod m) / m)).         */
/* phi_p = u1 of Philox counter (p, 0, 0, 5); s_i = floor(u1 * m) of counter */
/* (i, 0, 0, 6).  Written row-major like the Gaussian operator.             */
/* ------------------------------------------------------------------------ */
static double orc_u1(uint64_t seed, uint32_t stream, uint64_t col) {
  const uint32_t ctr[4] = {(uint32_t)col, (uint32_t)(col >> 32), 0u, stream};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return u52(w[0], w[1]);
}

int64_t orc_srft_row(uint64_t seed, uint64_t i, int64_t m) {
  int64_t s = (int64_t)floor(orc_u1(seed, 6u, i) * (double)m);
  return s < m ? s : m - 1;
}

double orc_srft_phase(uint64_t seed, uint64_t p) { return orc_u1(seed, 5u, p); }

void orc_srft_operator(int64_t l, int64_t m, uint64_t seed, double *out, int64_t ld) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < l; ++i) {
    const int64_t si = orc_srft_row(seed, (uint64_t)i, m);
    for (int64_t p = 0; p < m; ++p) {
      const int64_t r = (int64_t)(((__int128)si * p) % m);
      const double ang = ORC_TWO_PI * (orc_srft_phase(seed, (uint64_t)p) - (double)r / (double)m);
      out[2 * (i * ld + p)] = cos(ang);
      out[2 * (i * ld + p) + 1] = sin(ang);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Sketch, Sec. 2 randomization step with a Gaussian operator:               */
/*   Y(i, j) = sum_p G(i, p) A(p, j),  G l x m row-major (ld ldg),           */
/*   A m x n column-major (lda), Y l x n column-major (ldy).                 */
/* Straight sum over p = 0..m-1 in double.                                   */
/* ------------------------------------------------------------------------ */
void orc_sketch(int64_t m, int64_t n, int64_t l, const double *A, int64_t lda,
                const double *G, int64_t ldg, double *Y, int64_t ldy) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    const double *a = A + 2 * j * lda;
    for (int64_t i = 0; i < l; ++i) {
      const double *g = G + 2 * i * ldg;
      double sr = 0.0, si = 0.0;
      for (int64_t p = 0; p < m; ++p) {
        const double gr = g[2 * p], gi = g[2 * p + 1];
        const double ar = a[2 * p], ai = a[2 * p + 1];
        sr += gr * ar - gi * ai;
        si += gr * ai + gi * ar;
      }
      Y[2 * (i + j * ldy)] = sr;
      Y[2 * (i + j * ldy) + 1] = si;
    }
  }
}

/* Sketch of selected columns with G drawn on the fly from (seed, stream 0):
 * Ycols(:, c) = G * Acols(:, c) for c = 0..nc-1, Acols m x nc (ld lda).
 * Used to check sampled columns of a large sketch.                           */
void orc_sketch_seeded(int64_t m, int64_t nc, int64_t l, const double *Acols, int64_t lda,
                       uint64_t seed, double *Ycols, int64_t ldy) {
  double *G = (double *)malloc(sizeof(double) * 2 * (size_t)l * (size_t)m);
  orc_gaussian_rowmajor(l, m, seed, 0, G, m);
  orc_sketch(m, nc, l, Acols, lda, G, m, Ycols, ldy);
  free(G);
}

/* ------------------------------------------------------------------------ */
/* Greedy column selection and R, Sec. 2 approximate QR with the column      */
/* permutation, computed with the Gram-Schmidt of Sec. 3.2.                  */
/*                                                                           */
/* Step t picks the unselected column whose component orthogonal to the     */
/* columns picked so far has the largest 2-norm (first index wins an exact   */
/* tie), records gap_t = (best - second) / best, stops with ORC_ERR_RANK if */
/* best <= rank_tol * (best norm of step 0), and appends the normalised      */
/* residual of the winner, orthogonalised once more against Q (CGS2), to Q. */
/* Every unselected residual column then loses its component along the new  */
/* q, so residual norms are exact projections at every step.               */
/*                                                                           */
/* Outputs: J[0..k) pivot order; R = Q^H Y (k x n, column-major, ldr,        */
/* ORIGINAL column order); gaps[0..k).                                      */
/* ------------------------------------------------------------------------ */
static double cnorm2(const double *v, int64_t len) {
  double s = 0.0;
  for (int64_t i = 0; i < len; ++i) s += v[2 * i] * v[2 * i] + v[2 * i + 1] * v[2 * i + 1];
  return s;
}

/* dot = v^H w */
static void cdotc(const double *v, const double *w, int64_t len, double *dr, double *di) {
  double sr = 0.0, si = 0.0;
  for (int64_t i = 0; i < len; ++i) {
    sr += v[2 * i] * w[2 * i] + v[2 * i + 1] * w[2 * i + 1];
    si += v[2 * i] * w[2 * i + 1] - v[2 * i + 1] * w[2 * i];
  }
  *dr = sr; *di = si;
}

/* w -= v * (cr + i ci) */
static void caxpy_neg(double *w, const double *v, int64_t len, double cr, double ci) {
  for (int64_t i = 0; i < len; ++i) {
    w[2 * i] -= v[2 * i] * cr - v[2 * i + 1] * ci;
    w[2 * i + 1] -= v[2 * i] * ci + v[2 * i + 1] * cr;
  }
}

/* The same selection, optionally re-synchronised onto pivots chosen         */
/* elsewhere (Sec. 2 allows any permutation that brings the most weighted    */
/* columns to the front, so at a near-tie either candidate is a valid pick). */
/* With forced != NULL, step t takes column forced[t] (if >= 0) instead of   */
/* its own argmax, after recording, for that step:                           */
/*   argmax[t] = the oracle's own pick (greedy, lowest index on exact ties), */
/*   gaps[t]   = (best - second best) / best of the oracle's own norms,      */
/*   ratio[t]  = (trailing norm of the column taken) / best.                 */
/* A forced index that is out of range or already taken is an argument      */
/* error.  argmax and ratio may be NULL.                                     */
int orc_select_forced(int64_t l, int64_t n, int64_t k, const double *Y, int64_t ldy,
                      double rank_tol, const int64_t *forced, int64_t *J, double *R,
                      int64_t ldr, double *gaps, int64_t *argmax, double *ratio) {
  if (k < 1 || k > n || k > l || ldy < l || ldr < k) return ORC_ERR_ARG;
  double *res = (double *)malloc(sizeof(double) * 2 * (size_t)l * (size_t)n);
  double *Q = (double *)malloc(sizeof(double) * 2 * (size_t)l * (size_t)k);
  double *nu = (double *)malloc(sizeof(double) * (size_t)n);
  char *picked = (char *)calloc((size_t)n, 1);
  for (int64_t j = 0; j < n; ++j) memcpy(res + 2 * j * l, Y + 2 * j * ldy, sizeof(double) * 2 * l);
  double nu0 = 0.0;
  int status = ORC_OK;
  for (int64_t t = 0; t < k; ++t) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) nu[j] = picked[j] ? -1.0 : sqrt(cnorm2(res + 2 * j * l, l));
    int64_t best = -1;
    double b1 = -1.0, b2 = -1.0;
    for (int64_t j = 0; j < n; ++j) {
      if (picked[j]) continue;
      if (nu[j] > b1) { b2 = b1; b1 = nu[j]; best = j; }
      else if (nu[j] > b2) { b2 = nu[j]; }
    }
    if (t == 0) nu0 = b1;
    if (gaps) gaps[t] = (b2 < 0.0) ? 1.0 : (b1 > 0.0 ? (b1 - b2) / b1 : 0.0);
    if (argmax) argmax[t] = best;
    int64_t take = best;
    if (forced && forced[t] >= 0) {
      take = forced[t];
      if (take >= n || picked[take]) { status = ORC_ERR_ARG; break; }
    }
    if (ratio) ratio[t] = b1 > 0.0 ? nu[take] / b1 : 0.0;
    if (!(b1 > 0.0) || b1 <= rank_tol * nu0 || !(nu[take] > 0.0)) {
      status = ORC_ERR_RANK; J[t] = take; break;
    }
    J[t] = take;
    picked[take] = 1;
    double *q = Q + 2 * t * l;
    memcpy(q, res + 2 * take * l, sizeof(double) * 2 * l);
    /* second Gram-Schmidt pass against the existing basis */
    for (int64_t s = 0; s < t; ++s) {
      double cr, ci;
      cdotc(Q + 2 * s * l, q, l, &cr, &ci);
      caxpy_neg(q, Q + 2 * s * l, l, cr, ci);
    }
    const double qn = sqrt(cnorm2(q, l));
    for (int64_t i = 0; i < 2 * l; ++i) q[i] /= qn;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      if (picked[j]) continue;
      double cr, ci;
      cdotc(q, res + 2 * j * l, l, &cr, &ci);
      caxpy_neg(res + 2 * j * l, q, l, cr, ci);
    }
  }
  if (status == ORC_OK) {
    /* R = Q^H Y, original column order */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t t = 0; t < k; ++t) {
        double cr, ci;
        cdotc(Q + 2 * t * l, Y + 2 * j * ldy, l, &cr, &ci);
        R[2 * (t + j * ldr)] = cr;
        R[2 * (t + j * ldr) + 1] = ci;
      }
  }
  free(res); free(Q); free(nu); free(picked);
  return status;
}

int orc_select(int64_t l, int64_t n, int64_t k, const double *Y, int64_t ldy,
               double rank_tol, int64_t *J, double *R, int64_t ldr, double *gaps) {
  return orc_select_forced(l, n, k, Y, ldy, rank_tol, NULL, J, R, ldr, gaps, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Interpolation matrix, Sec. 2: solve R2 = R1 T with R1 = R(:, J) upper     */
/* triangular (only its upper triangle is read) by back substitution, one   */
/* column at a time, then P = [I T] in original column order:               */
/*   P(:, J[t]) = e_t,  P(:, j) = R1^{-1} R(:, j) for j not in J.            */
/* ------------------------------------------------------------------------ */
int orc_interp(int64_t n, int64_t k, const double *R, int64_t ldr, const int64_t *J,
               double *P, int64_t ldp) {
  if (k < 1 || k > n || ldr < k || ldp < k) return ORC_ERR_ARG;
  char *inJ = (char *)calloc((size_t)n, 1);
  for (int64_t t = 0; t < k; ++t) {
    if (J[t] < 0 || J[t] >= n || inJ[J[t]]) { free(inJ); return ORC_ERR_ARG; }
    inJ[J[t]] = 1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    double *p = P + 2 * j * ldp;
    if (inJ[j]) {
      for (int64_t t = 0; t < k; ++t) { p[2 * t] = 0.0; p[2 * t + 1] = 0.0; }
      continue;
    }
    for (int64_t t = k - 1; t >= 0; --t) {
      double sr = R[2 * (t + j * ldr)], si = R[2 * (t + j * ldr) + 1];
      for (int64_t s = t + 1; s < k; ++s) {
        const double *r = R + 2 * (t + J[s] * ldr);
        sr -= r[0] * p[2 * s] - r[1] * p[2 * s + 1];
        si -= r[0] * p[2 * s + 1] + r[1] * p[2 * s];
      }
      const double *d = R + 2 * (t + J[t] * ldr);
      const double den = d[0] * d[0] + d[1] * d[1];
      p[2 * t] = (sr * d[0] + si * d[1]) / den;
      p[2 * t + 1] = (si * d[0] - sr * d[1]) / den;
    }
  }
  for (int64_t t = 0; t < k; ++t) {
    double *p = P + 2 * J[t] * ldp;
    p[2 * t] = 1.0;
  }
  free(inJ);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* ||A - A(:, J) P||_2 by power iteration (the quantity of Table 5).         */
/* E = A - A(:,J) P is never formed: E x = A x~ with x~ = x - S_J (P x),     */
/* and E^H z = u - P^H u_J with u = A^H z, where S_J scatters entry t to      */
/* row J[t] and u_J gathers u at J.  Starting from x0 / ||x0||, step t        */
/* (t = 1..q) forms z = E x, records sigma_t = ||z||, and for t < q moves to  */
/* x = E^H z / ||E^H z||; it stops early, keeping sigma_t, if E^H z = 0.      */
/* All vectors and sums are binary128; A, P and x0 are exact doubles.        */
/* Returns sigma_q (or the early-stop value); hist[t-1] = sigma_t if hist.   */
/* ------------------------------------------------------------------------ */
typedef struct { __float128 re, im; } cq;

static __float128 qnorm(const cq *v, int64_t len) {
  __float128 s = 0;
  for (int64_t i = 0; i < len; ++i) s += v[i].re * v[i].re + v[i].im * v[i].im;
  return sqrtq(s);
}

int orc_residual(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                 const int64_t *J, const double *P, int64_t ldp, const double *x0, int q,
                 double *sigma, double *hist) {
  if (q < 1 || k < 0 || k > n || lda < m || (k > 0 && ldp < k)) return ORC_ERR_ARG;
  cq *x = (cq *)malloc(sizeof(cq) * (size_t)n);
  cq *xt = (cq *)malloc(sizeof(cq) * (size_t)n);
  cq *z = (cq *)malloc(sizeof(cq) * (size_t)m);
  cq *u = (cq *)malloc(sizeof(cq) * (size_t)n);
  cq *Px = (cq *)malloc(sizeof(cq) * (size_t)(k > 0 ? k : 1));
  for (int64_t j = 0; j < n; ++j) { x[j].re = x0[2 * j]; x[j].im = x0[2 * j + 1]; }
  {
    const __float128 nx = qnorm(x, n);
    for (int64_t j = 0; j < n; ++j) { x[j].re /= nx; x[j].im /= nx; }
  }
  double out = 0.0;
  for (int t = 1; t <= q; ++t) {
    /* x~ = x - S_J (P x) */
    for (int64_t s = 0; s < k; ++s) {
      __float128 sr = 0, si = 0;
      for (int64_t j = 0; j < n; ++j) {
        const __float128 pr = P[2 * (s + j * ldp)], pi = P[2 * (s + j * ldp) + 1];
        sr += pr * x[j].re - pi * x[j].im;
        si += pr * x[j].im + pi * x[j].re;
      }
      Px[s].re = sr; Px[s].im = si;
    }
    for (int64_t j = 0; j < n; ++j) xt[j] = x[j];
    for (int64_t s = 0; s < k; ++s) { xt[J[s]].re -= Px[s].re; xt[J[s]].im -= Px[s].im; }
    /* z = A x~ */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
      __float128 sr = 0, si = 0;
      for (int64_t j = 0; j < n; ++j) {
        const __float128 ar = A[2 * (i + j * lda)], ai = A[2 * (i + j * lda) + 1];
        sr += ar * xt[j].re - ai * xt[j].im;
        si += ar * xt[j].im + ai * xt[j].re;
      }
      z[i].re = sr; z[i].im = si;
    }
    const __float128 nz = qnorm(z, m);
    out = (double)nz;
    if (hist) hist[t - 1] = out;
    if (t == q) break;
    /* u = A^H z */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      __float128 sr = 0, si = 0;
      const double *a = A + 2 * j * lda;
      for (int64_t i = 0; i < m; ++i) {
        const __float128 ar = a[2 * i], ai = a[2 * i + 1];
        sr += ar * z[i].re + ai * z[i].im;
        si += ar * z[i].im - ai * z[i].re;
      }
      u[j].re = sr; u[j].im = si;
    }
    /* w = u - P^H u_J, stored in x */
    for (int64_t j = 0; j < n; ++j) {
      __float128 sr = u[j].re, si = u[j].im;
      for (int64_t s = 0; s < k; ++s) {
        const __float128 pr = P[2 * (s + j * ldp)], pi = P[2 * (s + j * ldp) + 1];
        const cq uj = u[J[s]];
        sr -= pr * uj.re + pi * uj.im;
        si -= pr * uj.im - pi * uj.re;
      }
      x[j].re = sr; x[j].im = si;
    }
    const __float128 nw = qnorm(x, n);
    if (nw == 0) { if (hist) for (int r = t; r < q; ++r) hist[r] = out; break; }
    for (int64_t j = 0; j < n; ++j) { x[j].re /= nw; x[j].im /= nw; }
  }
  *sigma = out;
  free(x); free(xt); free(z); free(u); free(Px);
  return ORC_OK;
}
