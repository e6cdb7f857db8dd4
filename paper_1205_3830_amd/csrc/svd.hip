// svd.hip -- the SVD of A built on its ID (Sec. 1 names fast SVDs among the
// ID's uses).  Given A (m x n), the skeleton J (k) and P (k x n) with
// A ~ A(:,J) P, return U (m x k), S (k, descending) and V (n x k) with
//   A(:,J) P = U diag(S) V^H
// exactly in exact arithmetic:
//   1. B = A(:, J) and its QR by shifted CholeskyQR3 (Fukaya, Kannan,
//      Nakatsukasa, Yamamoto, Yanagisawa, SISC 2020): a first Cholesky of
//      B^H B + s I with the shift s = 11 (mk + k(k+1)) u ||B||_F^2, then two
//      plain passes, so B = Q R_B, R_B = R3 R2 R1, for cond(B) up to about
//      1/u.  The Gram matrices and the products run on the FP64 matrix cores
//      (the sketch kernel), the Cholesky and the triangular inverse in one
//      workgroup;
//   2. M = R_B P (k x n), X = M^H (n x k);
//   3. one-sided Jacobi on X (Hestenes): column pairs rotated until mutually
//      orthogonal, round-robin pairing (k/2 pairs per launch, one launch per
//      round), the rotations accumulated in V_J (k x k).  No product M M^H is
//      formed, so small singular values keep their accuracy relative to M;
//   4. S_i = |X(:, i)|, V(:, i) = X(:, i) / S_i, U = Q V_J, sorted by S.
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
// workgroup.  R is written row-major (Rrm), R^-1 column-major (Rinv).  A
// pivot that is not positive sets *bad = 1 (and is replaced by 1 so that the
// kernel still ends with finite values); so does, when ident_tol > 0, an
// entry of W farther than ident_tol from the identity's (the last pass of
// CholeskyQR3 sees a Gram matrix within 5/64 of I whenever B has full
// numerical rank, far from it otherwise).
__global__ __launch_bounds__(256) void svd_chol_kernel(int64_t k, const double2 *__restrict__ W,
                                                       double shift_coef, double ident_tol,
                                                       double2 *__restrict__ Rrm,
                                                       double2 *__restrict__ Rinv, int *bad) {
  __shared__ double piv, shift;
  const int tid = threadIdx.x;
  if (ident_tol > 0.0) {
    for (int64_t e = tid; e < k * k; e += 256) {
      const double2 w = W[e];
      const double d = (e / k == e % k) ? w.x - 1.0 : w.x;
      if (!(sqrt(d * d + w.y * w.y) <= ident_tol)) *bad = 1;
    }
  }
  if (tid == 0) {
    double tr = 0.0;
    for (int64_t j = 0; j < k; ++j) tr += W[j * k + j].x;
    shift = shift_coef * tr;
  }
  for (int64_t e = tid; e < k * k; e += 256) Rrm[e] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int64_t j = 0; j < k; ++j) {
    if (tid == 0) {
      double d = W[j * k + j].x + shift;
      for (int64_t i = 0; i < j; ++i) {
        const double2 r = Rrm[i * k + j];
        d -= r.x * r.x + r.y * r.y;
      }
      if (!(d > 0.0)) {
        *bad = 1;
        d = 1.0;
      }
      piv = sqrt(d);
      Rrm[j * k + j] = make_double2(piv, 0.0);
    }
    __syncthreads();
    // R(j, c) = (W(j, c) - sum_{i<j} conj(R(i, j)) R(i, c)) / R(j, j), c > j
    for (int64_t c = j + 1 + tid; c < k; c += 256) {
      double2 s = W[c * k + j];
      for (int64_t i = 0; i < j; ++i) {
        const double2 a = Rrm[i * k + j], b = Rrm[i * k + c];
        s.x -= a.x * b.x + a.y * b.y;
        s.y -= a.x * b.y - a.y * b.x;
      }
      Rrm[j * k + c] = make_double2(s.x / piv, s.y / piv);
    }
    __syncthreads();
  }
  // R^-1, one column c per thread: R x = e_c by back substitution (x_i = 0
  // for i > c)
  for (int64_t c = tid; c < k; c += 256) {
    for (int64_t i = k - 1; i >= 0; --i) {
      double2 s = make_double2(0.0, 0.0);
      if (i <= c) {
        s.x = (i == c) ? 1.0 : 0.0;
        for (int64_t jj = i + 1; jj <= c; ++jj) {
          const double2 r = Rrm[i * k + jj], x = Rinv[c * k + jj];
          s.x -= r.x * x.x - r.y * x.y;
          s.y -= r.x * x.y + r.y * x.x;
        }
        const double d = Rrm[i * k + i].x;  // real diagonal
        s = make_double2(s.x / d, s.y / d);
      }
      Rinv[c * k + i] = s;
    }
  }
}

// C = A B of upper-triangular row-major k x k matrices (row-major result).
__global__ __launch_bounds__(256) void svd_trmul_kernel(int64_t k, const double2 *__restrict__ Am,
                                                        const double2 *__restrict__ Bm,
                                                        double2 *__restrict__ C) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < k * k;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / k, c = e - i * k;
    double sr = 0.0, si = 0.0;
    for (int64_t j = i; j <= c; ++j) {
      const double2 a = Am[i * k + j], b = Bm[j * k + c];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
    C[e] = make_double2(sr, si);
  }
}

// V_J = I (k x k column-major); the two flag words cleared.
__global__ void svd_init_kernel(int64_t k, double2 *V, int *flags) {
  const int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (g < 2) flags[g] = 0;
  for (int64_t e = g; e < k * k; e += int64_t(gridDim.x) * blockDim.x)
    V[e] = make_double2((e / k) == (e % k) ? 1.0 : 0.0, 0.0);
}

__global__ void svd_clear_kernel(int *flag) {
  if (threadIdx.x == 0) *flag = 0;
}

// Sums of four values over a 256-thread workgroup (every thread gets them).
RID_DEV void block_sum4(double &a, double &b, double &c, double &d, double *sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  d = wave_sum(d);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[4 * wave + 0] = a;
    sh[4 * wave + 1] = b;
    sh[4 * wave + 2] = c;
    sh[4 * wave + 3] = d;
  }
  __syncthreads();
  a = (sh[0] + sh[4]) + (sh[8] + sh[12]);
  b = (sh[1] + sh[5]) + (sh[9] + sh[13]);
  c = (sh[2] + sh[6]) + (sh[10] + sh[14]);
  d = (sh[3] + sh[7]) + (sh[11] + sh[15]);
}

// One round of one-sided Jacobi.  Workgroup b takes pair b of round r of the
// round-robin schedule on kk (even) players -- player kk-1 fixed, the others
// rotating; players >= k are padding.  With a = X(:, p), c = X(:, q) and
// gamma = a^H c, the pair is skipped when |gamma| <= tol |a| |c|; otherwise
// c is turned by the phase of gamma (so that a^H c becomes real) and a real
// rotation by the angle that zeroes it is applied to both columns, and the
// same transform to V_J's columns.  *rotated is set when any pair turned.
__global__ __launch_bounds__(256) void svd_jacobi_round_kernel(int64_t n, int64_t k, int64_t kk,
                                                               int64_t r, double2 *__restrict__ X,
                                                               int64_t ldx, double2 *__restrict__ V,
                                                               double tol, int *rotated) {
  __shared__ double sh[16];
  const int64_t b = blockIdx.x;
  int64_t p, q;
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
  if (q >= k) return;  // uniform over the workgroup
  double2 *xp = X + p * ldx, *xq = X + q * ldx;
  double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double2 a = xp[i], c = xq[i];
    al += a.x * a.x + a.y * a.y;
    be += c.x * c.x + c.y * c.y;
    gr += a.x * c.x + a.y * c.y;  // conj(a) c
    gi += a.x * c.y - a.y * c.x;
  }
  block_sum4(al, be, gr, gi, sh);
  const double g = sqrt(gr * gr + gi * gi);
  if (!(g > tol * sqrt(al) * sqrt(be))) return;  // uniform: every thread has the same sums
  if (threadIdx.x == 0) *rotated = 1;
  const double er = gr / g, ei = gi / g;  // e^{i phi} = gamma / |gamma|
  const double zeta = (be - al) / (2.0 * g);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
  for (int pass = 0; pass < 2; ++pass) {
    double2 *u = pass == 0 ? xp : V + p * k;
    double2 *w = pass == 0 ? xq : V + q * k;
    const int64_t len = pass == 0 ? n : k;
    for (int64_t i = threadIdx.x; i < len; i += 256) {
      const double2 a = u[i], c0 = w[i];
      const double2 c = make_double2(er * c0.x + ei * c0.y, er * c0.y - ei * c0.x);  // e^{-i phi} c0
      u[i] = make_double2(cs * a.x - sn * c.x, cs * a.y - sn * c.y);
      w[i] = make_double2(sn * a.x + cs * c.x, sn * a.y + cs * c.y);
    }
  }
}

// S_tmp(i) = |X(:, i)|, X(:, i) /= S_tmp(i) (one workgroup per column; a
// zero column stays zero).
__global__ __launch_bounds__(256) void svd_norm_kernel(int64_t n, double2 *__restrict__ X,
                                                       int64_t ldx, double *__restrict__ S) {
  __shared__ double sh[16];
  double2 *x = X + int64_t(blockIdx.x) * ldx;
  double s = 0.0, z0 = 0.0, z1 = 0.0, z2 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i].x * x[i].x + x[i].y * x[i].y;
  block_sum4(s, z0, z1, z2, sh);
  const double nrm = sqrt(s);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) x[i] = make_double2(x[i].x * inv, x[i].y * inv);
  if (threadIdx.x == 0) S[blockIdx.x] = nrm;
}

// Descending order of S (ties by index): column i goes to its rank; S, U's
// and V's columns are scattered there (one workgroup per column).
__global__ __launch_bounds__(256) void svd_scatter_kernel(int64_t m, int64_t n, int64_t k,
                                                          const double *__restrict__ Stmp,
                                                          const double2 *__restrict__ Ut,
                                                          const double2 *__restrict__ Xn,
                                                          double *__restrict__ S,
                                                          double2 *__restrict__ U, int64_t ldu,
                                                          double2 *__restrict__ V, int64_t ldv) {
  const int64_t i = blockIdx.x;
  const double si = Stmp[i];
  int64_t rank = 0;
  for (int64_t j = 0; j < k; ++j) {
    const double sj = Stmp[j];
    if (sj > si || (sj == si && j < i)) ++rank;
  }
  if (threadIdx.x == 0) S[rank] = si;
  for (int64_t p = threadIdx.x; p < m; p += 256) U[rank * ldu + p] = Ut[i * m + p];
  for (int64_t p = threadIdx.x; p < n; p += 256) V[rank * ldv + p] = Xn[i * n + p];
}

struct SvdWs {
  double2 *Qa, *Qb, *Qc, *Qt, *W, *R[3], *Rinv, *T, *RB, *M, *X, *VJ, *Ut;
  double *Stmp;
  int *flags;  // [0] Jacobi rotated, [1] Cholesky breakdown
  void *part;
};

template <class C>
SvdWs carve_svd(C &c, int64_t m, int64_t n, int64_t k) {
  SvdWs w;
  const size_t mk = size_t(m) * size_t(k), kk = size_t(k) * size_t(k), nk = size_t(n) * size_t(k);
  w.Qa = c.template take<double2>(mk);
  w.Qb = c.template take<double2>(mk);
  w.Qc = c.template take<double2>(mk);
  w.Qt = c.template take<double2>(mk);
  w.Ut = c.template take<double2>(mk);
  w.W = c.template take<double2>(kk);
  for (int i = 0; i < 3; ++i) w.R[i] = c.template take<double2>(kk);
  w.Rinv = c.template take<double2>(kk);
  w.T = c.template take<double2>(kk);
  w.RB = c.template take<double2>(kk);
  w.VJ = c.template take<double2>(kk);
  w.M = c.template take<double2>(nk);
  w.X = c.template take<double2>(nk);
  w.Stmp = c.template take<double>(size_t(k));
  w.flags = c.template take<int>(64);
  size_t part = 0;
  // the products: Gram (k x m)(m x k), Q R^-1 (m x k)(k x k), R_B P
  // (k x k)(k x n), Q V_J (m x k)(k x k)
  part = std::max(part, sketch_ws_bytes(RID_C128, RID_FP64, m, k, k));
  part = std::max(part, sketch_ws_bytes(RID_C128, RID_FP64, k, k, m));
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
  hipLaunchKernelGGL(svd_init_kernel, dim3(grid_for(k * k)), dim3(256), 0, st, k, w.VJ, w.flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == RID_C64)
    hipLaunchKernelGGL(svd_gather_kernel<float2>, dim3(grid_for(m * k)), dim3(256), 0, st, m,
                       n, k, static_cast<const float2 *>(A), lda, J, w.Qa);
  else
    hipLaunchKernelGGL(svd_gather_kernel<double2>, dim3(grid_for(m * k)), dim3(256), 0, st, m,
                       n, k, static_cast<const double2 *>(A), lda, J, w.Qa);
  e = hipGetLastError();
  // shifted CholeskyQR3: Q_{i+1} = Q_i R_{i+1}^-1 with R^H R = Q_i^H Q_i (+ s I)
  const double u = 0x1p-53;
  const double coef0 = 11.0 * (double(m) * double(k) + double(k) * double(k + 1)) * u;
  double2 *src = w.Qa, *dst = w.Qb;
  for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
    hipLaunchKernelGGL(svd_transpose_kernel<false>, dim3(grid_tiles(m, k)), dim3(256), 0, st, m,
                       k, src, m, w.Qt, k, w.Qc);
    e = hipGetLastError();
    if (e == hipSuccess) e = gemm(st, k, m, k, w.Qc, m, src, m, w.W, k, w.part);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(svd_chol_kernel, dim3(1), dim3(256), 0, st, k, w.W,
                         pass == 0 ? coef0 : 0.0, pass == 2 ? 0.5 : 0.0, w.R[pass], w.Rinv,
                         w.flags + 1);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = gemm(st, m, k, k, w.Qt, k, w.Rinv, k, dst, m, w.part);
    double2 *sw = src;
    src = dst;
    dst = sw;
  }
  // src = Q (m x k, orthonormal columns); R_B = R3 R2 R1
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_trmul_kernel, dim3(grid_for(k * k)), dim3(256), 0, st, k, w.R[2],
                       w.R[1], w.T);
    hipLaunchKernelGGL(svd_trmul_kernel, dim3(grid_for(k * k)), dim3(256), 0, st, k, w.T, w.R[0],
                       w.RB);
    e = hipGetLastError();
  }
  // M = R_B P (k x n), X = M^H (n x k)
  if (e == hipSuccess) e = gemm(st, k, k, n, w.RB, k, P, ldp, w.M, k, w.part);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_transpose_kernel<true>, dim3(grid_tiles(k, n)), dim3(256), 0, st, k, n,
                       w.M, k, w.X, n, static_cast<double2 *>(nullptr));
    e = hipGetLastError();
  }
  // the Cholesky status: a breakdown of the QR of B (a zero column)
  int h_flags[2] = {0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_flags, w.flags, sizeof(h_flags), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (h_flags[1]) {
    *rank_bad = 1;
    return hipSuccess;
  }
  // one-sided Jacobi on X (n x k, ld n); convergence read once per sweep
  const int64_t kk = (k % 2 == 0) ? k : k + 1;
  const double tol = sqrt(double(n)) * 0x1p-52;
  for (int sweep = 0; sweep < SVD_MAX_SWEEPS && k > 1; ++sweep) {
    hipLaunchKernelGGL(svd_clear_kernel, dim3(1), dim3(64), 0, st, w.flags);
    e = hipGetLastError();
    for (int64_t r = 0; r < kk - 1 && e == hipSuccess; ++r) {
      hipLaunchKernelGGL(svd_jacobi_round_kernel, dim3(static_cast<unsigned>(kk / 2)), dim3(256),
                         0, st, n, k, kk, r, w.X, n, w.VJ, tol, w.flags);
      e = hipGetLastError();
    }
    int h_rot = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h_rot, w.flags, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (sweeps_used) *sweeps_used = sweep + 1;
    if (!h_rot) break;
  }
  // S, V = the normalised columns of X, U = Q V_J, then sorted
  hipLaunchKernelGGL(svd_norm_kernel, dim3(static_cast<unsigned>(k)), dim3(256), 0, st, n, w.X, n,
                     w.Stmp);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_transpose_kernel<false>, dim3(grid_tiles(m, k)), dim3(256), 0, st, m,
                       k, src, m, w.Qt, k, static_cast<double2 *>(nullptr));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = gemm(st, m, k, k, w.Qt, k, w.VJ, k, w.Ut, m, w.part);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(svd_scatter_kernel, dim3(static_cast<unsigned>(k)), dim3(256), 0, st, m, n,
                       k, w.Stmp, w.Ut, w.X, S, U, ldu, V, ldv);
    e = hipGetLastError();
  }
  return e;
}
