// svd.hip -- the SVD of A built on its ID (Sec. 1 names fast SVDs among the
// ID's uses).  Given A (m x n), the skeleton J (k) and P (k x n) with
// A ~ A(:,J) P, return U (m x k), S (k, descending) and V (n x k) with
//   A(:,J) P = U diag(S) V^H
// exactly in exact arithmetic:
//   1. B = A(:, J) = Q R_B by shifted CholeskyQR3 (Fukaya, Kannan,
//      Nakatsukasa, Yamamoto, Yanagisawa, SISC 2020): a first Cholesky of
//      B^H B + s I with the shift s = 11 (mk + k(k+1)) u ||B||_F^2, then two
//      plain passes, R_B = R3 R2 R1; stable for cond(B) up to about 1/u.
//      The Gram matrices and the products run on the FP64 matrix cores (the
//      sketch kernel), the Cholesky and the triangular inverse in one
//      workgroup;
//   2. M = R_B P (k x n) and X = M^H (n x k) = Q_X R_X, the same QR;
//   3. one-sided Jacobi (Hestenes) on the k x k R_X, the QR-preconditioned
//      form of Jacobi on X (Drmac and Veselic): column pairs of R_X rotated
//      until mutually orthogonal, R_X Z = W diag(S), all sweeps in one
//      workgroup.  No product M M^H is formed, so small singular values keep
//      their accuracy relative to M;
//   4. then M = Z diag(S) (Q_X W)^H, so U = Q Z and V = Q_X W, sorted by S.
// All arithmetic is FP64 on complex128 operands (c64 A is widened).
#include <cmath>

#include "rid_internal.hpp"

namespace {

constexpr int SVD_KMAX = 256;
constexpr int SVD_MAX_SWEEPS = 60;

// B = A(:, J) (column-major m x k).  An index outside [0, n) gives a zero
// column (which the Cholesky then reports as a rank breakdown).
template <class TA>
__global__ __launch_bounds__(256) void svd_gather_kernel(int64_t m, int64_t n, int64_t k,
                                                         const TA *__restrict__ A, int64_t lda,
                                                         const int64_t *__restrict__ J,
                                                         double2 *__restrict__ B) {
  const int64_t total = m * k;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t t = e / m;
    const int64_t p = e - t * m;
    const int64_t j = J[t];
    B[e] = (j >= 0 && j < n) ? to_d2(A[j * lda + p]) : make_double2(0.0, 0.0);
  }
}

// in: rows x cols, column-major (ldin).  out_t(c, r) = in(r, c) (conjugated
// when CONJ_T), out_t column-major (cols x rows, ldt); out_c (optional) =
// conj(in) in in's layout.  32 x 32 tiles staged in LDS so that both the
// reads and the transposed writes are coalesced.
template <bool CONJ_T>
__global__ __launch_bounds__(256) void svd_transpose_kernel(int64_t rows, int64_t cols,
                                                            const double2 *__restrict__ in,
                                                            int64_t ldin, double2 *__restrict__ out_t,
                                                            int64_t ldt, double2 *__restrict__ out_c) {
  __shared__ double2 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t tr = (rows + 31) / 32, tc = (cols + 31) / 32;
  for (int64_t t = blockIdx.x; t < tr * tc; t += gridDim.x) {
    const int64_t r0 = (t % tr) * 32, c0 = (t / tr) * 32;
    const int64_t r = r0 + tx;
    for (int j = ty; j < 32; j += 8) {
      const int64_t c = c0 + j;
      double2 v = make_double2(0.0, 0.0);
      if (r < rows && c < cols) {
        v = in[c * ldin + r];
        if (out_c) out_c[c * ldin + r] = make_double2(v.x, -v.y);
      }
      tile[j][tx] = v;
    }
    __syncthreads();
    const int64_t c = c0 + tx;
    for (int j = ty; j < 32; j += 8) {
      const int64_t rr = r0 + j;
      if (rr < rows && c < cols) {
        double2 v = tile[tx][j];
        if (CONJ_T) v.y = -v.y;
        out_t[rr * ldt + c] = v;
      }
    }
    __syncthreads();
  }
}

// Upper Cholesky W + s I = R^H R of the k x k Hermitian W (column-major,
// ld k, upper triangle read), s = shift_coef * trace(W), and R^-1, in one
// workgroup of 1024 threads, both right-looking: after pivot j the trailing
// Schur complement (Sm) loses the outer product of row j of R; R^-1 is
// built in Sm from its last row up, each finished row j subtracting
// R(i, j) R^-1(j, :) from the rows i < j still open.  R is written row-major
// (Rrm), R^-1 column-major (Rinv).  Sm (k x k) and vec (k) are the working
// arrays, in LDS or global memory as the caller chooses.  A pivot that is
// not positive sets *bad = 1 (and is replaced by 1 so that the kernel still
// ends with finite values); so does, when ident_tol > 0, an entry of W
// farther than ident_tol from the identity's (the last pass of CholeskyQR3
// sees a Gram matrix within 5/64 of I whenever its input has full
// numerical rank).
RID_DEV void chol_body(int64_t k, const double2 *__restrict__ W, double shift_coef,
                       double ident_tol, double2 *__restrict__ Rrm, double2 *__restrict__ Rinv,
                       double2 *Sm, double2 *vec, double *red, double *piv_s, int *bad) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  if (ident_tol > 0.0) {
    for (int64_t e = tid; e < k * k; e += nt) {
      const double2 w = W[e];
      const double d = (e / k == e % k) ? w.x - 1.0 : w.x;
      if (!(sqrt(d * d + w.y * w.y) <= ident_tol)) *bad = 1;
    }
  }
  double tr = 0.0;
  for (int64_t j = tid; j < k; j += nt) tr += W[j * k + j].x;
  tr = wave_sum(tr);
  if ((tid & 63) == 0) red[tid >> 6] = tr;
  __syncthreads();
  double total = 0.0;
  for (int i = 0; i < (nt >> 6); ++i) total += red[i];
  const double shift = shift_coef * total;
  for (int64_t e = tid; e < k * k; e += nt) {
    const double2 w = W[e];
    Sm[e] = (e / k) == (e % k) ? make_double2(w.x + shift, 0.0) : w;
    Rrm[e] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int64_t j = 0; j < k; ++j) {
    if (tid == 0) {
      double d = Sm[j * k + j].x;
      if (!(d > 0.0)) {
        *bad = 1;
        d = 1.0;
      }
      *piv_s = sqrt(d);
      Rrm[j * k + j] = make_double2(*piv_s, 0.0);
    }
    __syncthreads();
    const double piv = *piv_s;
    for (int64_t c = j + 1 + tid; c < k; c += nt) {
      const double2 v = Sm[c * k + j];
      const double2 r = make_double2(v.x / piv, v.y / piv);
      Rrm[j * k + c] = r;
      vec[c] = r;
    }
    __syncthreads();
    // Sm(a, c) -= conj(R(j, a)) R(j, c), j < a <= c
    const int64_t w = k - j - 1;
    for (int64_t e = tid; e < w * w; e += nt) {
      const int64_t a = j + 1 + e % w, c = j + 1 + e / w;
      if (a > c) continue;
      const double2 x = vec[a], y = vec[c];
      double2 s = Sm[c * k + a];
      s.x -= x.x * y.x + x.y * y.y;
      s.y -= x.x * y.y - x.y * y.x;
      Sm[c * k + a] = s;
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < k * k; e += nt)
    Sm[e] = make_double2((e / k) == (e % k) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int64_t jj = k - 1; jj >= 0; --jj) {
    const double d = Rrm[jj * k + jj].x;  // real diagonal
    for (int64_t c = jj + tid; c < k; c += nt) {
      const double2 v = Sm[c * k + jj];
      Sm[c * k + jj] = make_double2(v.x / d, v.y / d);
    }
    for (int64_t i = tid; i < jj; i += nt) vec[i] = Rrm[i * k + jj];
    __syncthreads();
    // T(i, c) -= R(i, jj) R^-1(jj, c), i < jj <= c
    const int64_t cols = k - jj;
    for (int64_t e = tid; e < jj * cols; e += nt) {
      const int64_t i = e % jj, c = jj + e / jj;
      const double2 r = vec[i], x = Sm[c * k + jj];
      double2 t = Sm[c * k + i];
      t.x -= r.x * x.x - r.y * x.y;
      t.y -= r.x * x.y + r.y * x.x;
      Sm[c * k + i] = t;
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < k * k; e += nt) Rinv[e] = Sm[e];
}

// Working arrays in global memory (any k <= 256).
__global__ __launch_bounds__(1024) void svd_chol_kernel(int64_t k, const double2 *__restrict__ W,
                                                        double shift_coef, double ident_tol,
                                                        double2 *__restrict__ Rrm,
                                                        double2 *__restrict__ Rinv,
                                                        double2 *__restrict__ Sch,
                                                        double2 *__restrict__ vec, int *bad) {
  __shared__ double red[16], piv_s;
  chol_body(k, W, shift_coef, ident_tol, Rrm, Rinv, Sch, vec, red, &piv_s, bad);
}

// Working arrays in LDS for k <= 100 (156 KB of the 160 KB one workgroup
// may hold on gfx950).
__global__ __launch_bounds__(1024) void svd_chol_lds_kernel(int64_t k,
                                                            const double2 *__restrict__ W,
                                                            double shift_coef, double ident_tol,
                                                            double2 *__restrict__ Rrm,
                                                            double2 *__restrict__ Rinv, int *bad) {
  __shared__ double2 sm[100 * 100];
  __shared__ double2 vec[100];
  __shared__ double red[16], piv_s;
  chol_body(k, W, shift_coef, ident_tol, Rrm, Rinv, sm, vec, red, &piv_s, bad);
}

// C = A B of upper-triangular row-major k x k matrices, C row-major or (with
// col_major) column-major.
__global__ __launch_bounds__(256) void svd_trmul_kernel(int64_t k, const double2 *__restrict__ Am,
                                                        const double2 *__restrict__ Bm,
                                                        double2 *__restrict__ C, int col_major) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < k * k;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / k, c = e - i * k;
    double sr = 0.0, si = 0.0;
    for (int64_t j = i; j <= c; ++j) {
      const double2 a = Am[i * k + j], b = Bm[j * k + c];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
    C[col_major ? c * k + i : e] = make_double2(sr, si);
  }
}

// Z = I (k x k column-major); the two flag words cleared.
__global__ void svd_init_kernel(int64_t k, double2 *Z, int *flags) {
  const int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (g < 2) flags[g] = 0;
  for (int64_t e = g; e < k * k; e += int64_t(gridDim.x) * blockDim.x)
    Z[e] = make_double2((e / k) == (e % k) ? 1.0 : 0.0, 0.0);
}

// Round r of the round-robin schedule on kk (even) players -- player kk-1
// fixed, the others rotating: pair b of the round, p < q.  Players >= k are
// padding.  Every pair of players meets once in kk - 1 rounds, and the
// pairs of one round are disjoint.
RID_DEV void rr_pair(int64_t kk, int64_t r, int64_t b, int64_t &p, int64_t &q) {
  if (b == 0) {
    p = r;
    q = kk - 1;
  } else {
    p = (r + b) % (kk - 1);
    q = (r - b + kk - 1) % (kk - 1);
  }
  if (p > q) {
    const int64_t sw = p;
    p = q;
    q = sw;
  }
}

// The rotation of one pair: c is turned by the phase e^{-i phi}
// (er - i ei) and then (a, c) by the real rotation (cs, sn).
RID_DEV void turn(double cs, double sn, double er, double ei, double2 a, double2 c0, double2 &na,
                  double2 &nc) {
  const double2 c = make_double2(er * c0.x + ei * c0.y, er * c0.y - ei * c0.x);
  na = make_double2(cs * a.x - sn * c.x, cs * a.y - sn * c.y);
  nc = make_double2(sn * a.x + cs * c.x, sn * a.y + cs * c.y);
}

// One-sided Jacobi on the columns of R (k x k column-major), all sweeps in
// one workgroup of 1024 threads.  A sweep is kk - 1 rounds (kk = k rounded
// up to even) whose kk/2 disjoint pairs run at once, G lanes per pair.
// With a = R(:, p), c = R(:, q) and gamma = a^H c, a pair is left alone when
// |gamma|^2 <= tol^2 |a|^2 |c|^2; otherwise c is turned by the phase of
// gamma (so that a^H c becomes real) and a real rotation by the angle that
// zeroes it, t = tan(angle), is applied to both columns.  The squared
// column norms live in nrm (LDS): computed at the start of each sweep, then
// updated as |a|^2 - t |gamma| and |c|^2 + t |gamma| after each rotation
// (exact in exact arithmetic: the rotation preserves the trace of the 2 x 2
// Gram matrix and zeroes its off-diagonal).  The same transforms make Z:
// with REC false they are applied to the columns of Zw in place (and the
// rounds end with a full barrier); with REC true each pair's transform is
// written to rec (identity when the pair is left alone) for
// svd_rot_apply_kernel, and, R being in LDS, the rounds end with an
// LDS-only barrier.  Sweeps stop after one without a rotation, at most
// max_sweeps; returns their number.
template <int G, bool REC>
RID_DEV int jacobi_sweeps(int64_t k, double2 *Rw, double2 *Zw, double2 *__restrict__ rec,
                          double tol, int max_sweeps, double *nrm, int *rotated) {
  const int tid = threadIdx.x;
  const int grp = tid / G, gl = tid % G;
  const int ngrp = blockDim.x / G;
  const int64_t kk = (k % 2 == 0) ? k : k + 1;
  const double tol2 = tol * tol;
  auto barrier = [] {
    if (REC) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
      __syncthreads();
    }
  };
  int sweep = 0;
  while (sweep < max_sweeps) {
    if (tid == 0) *rotated = 0;
    for (int64_t c = grp; c < k; c += ngrp) {  // uniform within the group
      const double2 *x = Rw + c * k;
      double s = 0.0;
      for (int64_t i = gl; i < k; i += G) s += x[i].x * x[i].x + x[i].y * x[i].y;
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
      if (gl == 0) nrm[c] = s;
    }
    barrier();
    for (int64_t r = 0; r < kk - 1; ++r) {
      for (int64_t b = grp; b < kk / 2; b += ngrp) {  // uniform within the group
        int64_t p, q;
        rr_pair(kk, r, b, p, q);
        if (q >= k) continue;
        double2 *xp = Rw + p * k, *xq = Rw + q * k;
        double gr = 0.0, gi = 0.0;
        for (int64_t i = gl; i < k; i += G) {
          const double2 a = xp[i], c = xq[i];
          gr += a.x * c.x + a.y * c.y;  // conj(a) c
          gi += a.x * c.y - a.y * c.x;
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
          gr += __shfl_xor(gr, o, G);
          gi += __shfl_xor(gi, o, G);
        }
        const double al = nrm[p], be = nrm[q];
        const double g2 = gr * gr + gi * gi;
        const bool go = g2 > tol2 * al * be;  // uniform within the group
        double cs = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
        double t = 0.0, g = 0.0;
        if (go) {
          g = sqrt(g2);
          const double rg = 1.0 / g;
          er = gr * rg;  // e^{i phi} = gamma / |gamma|
          ei = gi * rg;
          const double zeta = (be - al) * (0.5 * rg);
          t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          cs = 1.0 / sqrt(1.0 + t * t);
          sn = cs * t;
        }
        if (REC && gl == 0) {
          double2 *o = rec + 2 * ((int64_t(sweep) * (kk - 1) + r) * (kk / 2) + b);
          o[0] = make_double2(cs, sn);
          o[1] = make_double2(er, ei);
        }
        if (!go) continue;
        if (gl == 0) {
          *rotated = 1;
          nrm[p] = al - t * g;
          nrm[q] = be + t * g;
        }
        for (int64_t i = gl; i < k; i += G) turn(cs, sn, er, ei, xp[i], xq[i], xp[i], xq[i]);
        if (!REC) {
          double2 *zp = Zw + p * k, *zq = Zw + q * k;
          for (int64_t i = gl; i < k; i += G) turn(cs, sn, er, ei, zp[i], zq[i], zp[i], zq[i]);
        }
      }
      barrier();
    }
    ++sweep;
    const int any = *rotated;
    barrier();  // every thread has read the flag before the next reset
    if (!any) break;
  }
  return sweep;
}

// R and Z in global memory (any k <= 256).
template <int G>
__global__ __launch_bounds__(1024) void svd_jacobi_kernel(int64_t k, double2 *__restrict__ R,
                                                          double2 *__restrict__ Z, double tol,
                                                          int max_sweeps, int *sweeps) {
  __shared__ int rotated;
  __shared__ double nrm[256];
  const int sw = jacobi_sweeps<G, false>(k, R, Z, nullptr, tol, max_sweeps, nrm, &rotated);
  if (threadIdx.x == 0) *sweeps = sw;
}

// R and Z both staged in LDS (k <= 64: 128 KB).
__global__ __launch_bounds__(1024) void svd_jacobi_lds_kernel(int64_t k, double2 *__restrict__ R,
                                                              double2 *__restrict__ Z, double tol,
                                                              int max_sweeps, int *sweeps) {
  __shared__ double2 rs[64 * 64];
  __shared__ double2 zs[64 * 64];
  __shared__ double nrm[64];
  __shared__ int rotated;
  for (int64_t e = threadIdx.x; e < k * k; e += blockDim.x) {
    rs[e] = R[e];
    zs[e] = Z[e];
  }
  __syncthreads();
  const int sw = jacobi_sweeps<8, false>(k, rs, zs, nullptr, tol, max_sweeps, nrm, &rotated);
  for (int64_t e = threadIdx.x; e < k * k; e += blockDim.x) {
    R[e] = rs[e];
    Z[e] = zs[e];
  }
  if (threadIdx.x == 0) *sweeps = sw;
}

// R staged in LDS (k <= 100: 156 KB of the 160 KB one workgroup may hold on
// gfx950); the transforms go to rec for svd_rot_apply_kernel.
__global__ __launch_bounds__(1024) void svd_jacobi_rec_kernel(int64_t k, double2 *__restrict__ R,
                                                              double2 *__restrict__ rec,
                                                              double tol, int max_sweeps,
                                                              int *sweeps) {
  __shared__ double2 rs[100 * 100];
  __shared__ double nrm[100];
  __shared__ int rotated;
  for (int64_t e = threadIdx.x; e < k * k; e += blockDim.x) rs[e] = R[e];
  __syncthreads();
  const int sw = jacobi_sweeps<8, true>(k, rs, nullptr, rec, tol, max_sweeps, nrm, &rotated);
  __syncthreads();
  for (int64_t e = threadIdx.x; e < k * k; e += blockDim.x) R[e] = rs[e];
  if (threadIdx.x == 0) *sweeps = sw;
}

// Z = the product of the transforms in rec (from svd_jacobi_rec_kernel, k <=
// 100, *nsweeps sweeps), Z column-major.  Row i of Z is e_i^T times the
// transforms in order, and rows do not interact: one wavefront per row,
// lane b taking pair b of each round (kk/2 <= 50 lanes), the row in LDS,
// the records read D rounds ahead.
__global__ __launch_bounds__(1024) void svd_rot_apply_kernel(int64_t k,
                                                             const double2 *__restrict__ rec,
                                                             const int *__restrict__ nsweeps,
                                                             double2 *__restrict__ Z) {
  constexpr int D = 4;
  __shared__ double2 zrow[16][100];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = int64_t(blockIdx.x) * 16 + wave;
  if (i >= k) return;  // the whole wavefront; no workgroup barrier follows
  double2 *z = zrow[wave];
  for (int64_t c = lane; c < k; c += 64) z[c] = make_double2(c == i ? 1.0 : 0.0, 0.0);
  const int64_t kk = (k % 2 == 0) ? k : k + 1;
  const int64_t np = kk / 2, nr = kk - 1;
  const int64_t total = int64_t(*nsweeps) * nr;
  const bool mine = lane < np;
  double2 ra[D], rb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const bool ok = mine && d < total;
    ra[d] = ok ? rec[2 * (d * np + lane)] : make_double2(1.0, 0.0);
    rb[d] = ok ? rec[2 * (d * np + lane) + 1] : make_double2(1.0, 0.0);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  for (int64_t t0 = 0; t0 < total; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t t = t0 + d;
      if (t >= total) break;
      const double2 ca = ra[d], cb = rb[d];
      const int64_t tn = t + D;
      if (mine && tn < total) {
        ra[d] = rec[2 * (tn * np + lane)];
        rb[d] = rec[2 * (tn * np + lane) + 1];
      }
      int64_t p, q;
      rr_pair(kk, t % nr, lane, p, q);
      if (mine && q < k) turn(ca.x, ca.y, cb.x, cb.y, z[p], z[q], z[p], z[q]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    }
  }
  for (int64_t c = lane; c < k; c += 64) Z[c * k + i] = z[c];
}

// S = the column norms of R (k x k) in descending order (ties by index);
// column i of R, normalised, and of Z go to column rank(i) of Ws and Zs
// (a zero column stays zero).  One workgroup, k <= 256.
__global__ __launch_bounds__(256) void svd_sort_kernel(int64_t k, const double2 *__restrict__ R,
                                                       const double2 *__restrict__ Z,
                                                       double *__restrict__ S,
                                                       double2 *__restrict__ Ws,
                                                       double2 *__restrict__ Zs) {
  __shared__ double nrm[256];
  __shared__ int rank[256];
  const int tid = threadIdx.x;
  if (tid < k) {
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) {
      const double2 v = R[tid * k + i];
      s += v.x * v.x + v.y * v.y;
    }
    nrm[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid < k) {
    const double si = nrm[tid];
    int rk = 0;
    for (int j = 0; j < k; ++j) {
      const double sj = nrm[j];
      if (sj > si || (sj == si && j < tid)) ++rk;
    }
    rank[tid] = rk;
    S[rk] = si;
  }
  __syncthreads();
  for (int64_t e = tid; e < k * k; e += 256) {
    const int64_t i = e / k, r = e - i * k;
    const int64_t o = int64_t(rank[i]) * k + r;
    const double inv = nrm[i] > 0.0 ? 1.0 / nrm[i] : 0.0;
    const double2 v = R[e];
    Ws[o] = make_double2(v.x * inv, v.y * inv);
    Zs[o] = Z[e];
  }
}

struct SvdWs {
  double2 *Qa, *Qb, *Xa, *Xb, *Qc, *Qt, *M;
  double2 *W, *Sch, *Rinv, *T, *RB, *RX, *Z, *Zs, *Ws, *vec;
  double2 *rec;  // Jacobi transforms (two double2 per pair and round)
  double2 *R[6];  // the R factors of the two CholeskyQR3 runs
  int *flags;     // [0] Jacobi sweeps, [1] Cholesky breakdown
  void *part;
};

template <class C>
SvdWs carve_svd(C &c, int64_t m, int64_t n, int64_t k) {
  SvdWs w;
  const size_t mk = size_t(m) * size_t(k), kk = size_t(k) * size_t(k), nk = size_t(n) * size_t(k);
  const size_t big = std::max(mk, nk);
  w.Qa = c.template take<double2>(mk);
  w.Qb = c.template take<double2>(mk);
  w.Xa = c.template take<double2>(nk);
  w.Xb = c.template take<double2>(nk);
  w.Qc = c.template take<double2>(big);
  w.Qt = c.template take<double2>(big);
  w.M = c.template take<double2>(nk);
  double2 **small[] = {&w.W, &w.Sch, &w.Rinv, &w.T, &w.RB, &w.RX, &w.Z, &w.Zs, &w.Ws};
  for (double2 **p : small) *p = c.template take<double2>(kk);
  for (int i = 0; i < 6; ++i) w.R[i] = c.template take<double2>(kk);
  w.vec = c.template take<double2>(size_t(k));
  const size_t kke = size_t(k % 2 == 0 ? k : k + 1);
  w.rec = c.template take<double2>(k <= 100 ? 2 * size_t(SVD_MAX_SWEEPS) * (kke - 1) * (kke / 2)
                                            : 1);
  w.flags = c.template take<int>(64);
  size_t part = 0;
  // the products: Gram (k x rows)(rows x k), Q R^-1 (rows x k)(k x k) for
  // rows = m and n, and R_B P (k x k)(k x n)
  for (int64_t rows : {m, n}) {
    part = std::max(part, sketch_ws_bytes(RID_C128, RID_FP64, rows, k, k));
    part = std::max(part, sketch_ws_bytes(RID_C128, RID_FP64, k, k, rows));
  }
  part = std::max(part, sketch_ws_bytes(RID_C128, RID_FP64, k, n, k));
  w.part = c.template take<char>(part);
  return w;
}

unsigned grid_for(int64_t total, int64_t per = 256) {
  int64_t b = (total + per - 1) / per;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

unsigned grid_tiles(int64_t rows, int64_t cols) {
  const int64_t t = ((rows + 31) / 32) * ((cols + 31) / 32);
  return static_cast<unsigned>(t < 1 ? 1 : (t > 65536 ? 65536 : t));
}

// out (rows x cols, column-major, ldo) = Xrm (rows x inner, row-major, ldx)
//                                        Z (inner x cols, column-major, ldz)
hipError_t gemm(hipStream_t st, int64_t rows, int64_t inner, int64_t cols, const double2 *Xrm,
                int64_t ldx, const double2 *Z, int64_t ldz, double2 *out, int64_t ldo,
                void *part) {
  return launch_sketch(st, RID_C128, RID_FP64, inner, cols, rows, Z, ldz, Xrm, ldx, out, ldo, part,
                       nullptr);
}

// Shifted CholeskyQR3 of src (rows x k, column-major, ld rows): Q = src R^-1
// with R = R3 R2 R1 (upper triangular) written to Rout (row-major, or
// column-major with rout_col_major).  src and tmp are overwritten; *q is
// whichever of them holds Q.
hipError_t cholqr3(hipStream_t st, int64_t rows, int64_t k, double2 *src, double2 *tmp,
                   double2 *const *R3, double2 *Rout, int rout_col_major, const SvdWs &w,
                   double2 **q) {
  const double u = 0x1p-53;
  const double coef0 = 11.0 * (double(rows) * double(k) + double(k) * double(k + 1)) * u;
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
    hipLaunchKernelGGL(svd_transpose_kernel<false>, dim3(grid_tiles(rows, k)), dim3(256), 0, st,
                       rows, k, src, rows, w.Qt, k, w.Qc);
    e = hipGetLastError();
    if (e == hipSuccess) e = gemm(st, k, rows, k, w.Qc, rows, src, rows, w.W, k, w.part);
    if (e == hipSuccess) {
      const double shift = pass == 0 ? coef0 : 0.0, ident = pass == 2 ? 0.5 : 0.0;
      if (k <= 100)
        hipLaunchKernelGGL(svd_chol_lds_kernel, dim3(1), dim3(1024), 0, st, k, w.W, shift, ident,
                           R3[pass], w.Rinv, w.flags + 1);
      else
        hipLaunchKernelGGL(svd_chol_kernel, dim3(1), dim3(1024), 0, st, k, w.W, shift, ident,
                           R3[pass], w.Rinv, w.Sch, w.vec, w.flags + 1);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = gemm(st, rows, k, k, w.Qt, k, w.Rinv, k, tmp, rows, w.part);
    double2 *sw = src;
    src = tmp;
    tmp = sw;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_trmul_kernel, dim3(grid_for(k * k)), dim3(256), 0, st, k, R3[2], R3[1],
                       w.T, 0);
    hipLaunchKernelGGL(svd_trmul_kernel, dim3(grid_for(k * k)), dim3(256), 0, st, k, w.T, R3[0],
                       Rout, rout_col_major);
    e = hipGetLastError();
  }
  *q = src;
  return e;
}

}  // namespace

bool svd_supported(int64_t k) { return k >= 1 && k <= SVD_KMAX; }

size_t svd_ws_bytes(int64_t m, int64_t n, int64_t k) {
  WsCarve c(nullptr);
  carve_svd(c, m, n, k);
  return c.off + 256;
}

hipError_t launch_svd(hipStream_t st, rid_dtype dtype, int64_t m, int64_t n, int64_t k,
                      const void *A, int64_t lda, const int64_t *J, const double2 *P, int64_t ldp,
                      double2 *U, int64_t ldu, double *S, double2 *V, int64_t ldv, void *ws,
                      int *rank_bad, int *sweeps_used) {
  WsCarve c(ws);
  const SvdWs w = carve_svd(c, m, n, k);
  *rank_bad = 0;
  if (sweeps_used) *sweeps_used = 0;
  hipLaunchKernelGGL(svd_init_kernel, dim3(grid_for(k * k)), dim3(256), 0, st, k, w.Z, w.flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == RID_C64)
    hipLaunchKernelGGL(svd_gather_kernel<float2>, dim3(grid_for(m * k)), dim3(256), 0, st, m,
                       n, k, static_cast<const float2 *>(A), lda, J, w.Qa);
  else
    hipLaunchKernelGGL(svd_gather_kernel<double2>, dim3(grid_for(m * k)), dim3(256), 0, st, m,
                       n, k, static_cast<const double2 *>(A), lda, J, w.Qa);
  e = hipGetLastError();
  // B = Q R_B
  double2 *Q = nullptr, *QX = nullptr;
  if (e == hipSuccess) e = cholqr3(st, m, k, w.Qa, w.Qb, w.R, w.RB, 0, w, &Q);
  // M = R_B P (k x n), X = M^H (n x k) = Q_X R_X
  if (e == hipSuccess) e = gemm(st, k, k, n, w.RB, k, P, ldp, w.M, k, w.part);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_transpose_kernel<true>, dim3(grid_tiles(k, n)), dim3(256), 0, st, k, n,
                       w.M, k, w.Xa, n, static_cast<double2 *>(nullptr));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = cholqr3(st, n, k, w.Xa, w.Xb, w.R + 3, w.RX, 1, w, &QX);
  // R_X Z = W diag(S), sorted
  if (e == hipSuccess) {
    const double tol = sqrt(double(k)) * 0x1p-52;
    if (k <= 64) {
      hipLaunchKernelGGL(svd_jacobi_lds_kernel, dim3(1), dim3(1024), 0, st, k, w.RX, w.Z, tol,
                         SVD_MAX_SWEEPS, w.flags);
    } else if (k <= 100) {
      hipLaunchKernelGGL(svd_jacobi_rec_kernel, dim3(1), dim3(1024), 0, st, k, w.RX, w.rec, tol,
                         SVD_MAX_SWEEPS, w.flags);
      hipLaunchKernelGGL(svd_rot_apply_kernel, dim3(static_cast<unsigned>((k + 15) / 16)),
                         dim3(1024), 0, st, k, w.rec, w.flags, w.Z);
    } else {
      hipLaunchKernelGGL(svd_jacobi_kernel<8>, dim3(1), dim3(1024), 0, st, k, w.RX, w.Z, tol,
                         SVD_MAX_SWEEPS, w.flags);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_sort_kernel, dim3(1), dim3(256), 0, st, k, w.RX, w.Z, S, w.Ws, w.Zs);
    e = hipGetLastError();
  }
  // U = Q Z, V = Q_X W (written in place into the caller's outputs)
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_transpose_kernel<false>, dim3(grid_tiles(m, k)), dim3(256), 0, st, m,
                       k, Q, m, w.Qt, k, static_cast<double2 *>(nullptr));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = gemm(st, m, k, k, w.Qt, k, w.Zs, k, U, ldu, w.part);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_transpose_kernel<false>, dim3(grid_tiles(n, k)), dim3(256), 0, st, n,
                       k, QX, n, w.Qt, k, static_cast<double2 *>(nullptr));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = gemm(st, n, k, k, w.Qt, k, w.Ws, k, V, ldv, w.part);
  int h_flags[2] = {0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_flags, w.flags, sizeof(h_flags), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (sweeps_used) *sweeps_used = h_flags[0];
  *rank_bad = h_flags[1] != 0;
  return hipSuccess;
}
