// residual.hip -- the error ||A - A(:,J) P||_2 of Table 5, estimated by power
// iteration on E = A - A(:,J) P without forming E:
//   E x   = A x~,           x~ = x - S_J (P x)       (S_J scatters to rows J)
//   E^H z = u - P^H u_J,    u  = A^H z
// E is ~1e-10 of A, so both products cancel almost completely.  Every sum
// over A is therefore compensated (Ogita-Rump-Oishi Dot2: exact products by
// FMA, TwoSum for the running sum, errors collected in a second double) and
// x~, u and the P-corrections are carried as double-double pairs.
//
// The two passes over A are the HBM-bound kernels of the whole ID; both read
// A with non-temporal loads (A is touched once per pass):
//   ax_partial : z = A x~ ; a workgroup streams a 512-row slab of a range of
//                columns (each column slab is one contiguous 8 KB read).
//   ahz_partial: u = A^H z ; a workgroup stages a 2048-row chunk of z in LDS
//                and each wave streams 8 columns of that chunk (32 KB
//                contiguous reads each), reducing in registers then across
//                lanes.
// Partial sums over column splits (resp. row splits) are reduced in a fixed
// order by separate kernels, so results are bitwise reproducible.
#include "rid_internal.hpp"

namespace {

constexpr int AX_ROWS = 512;   // rows per ax workgroup (2 per thread)
constexpr int AHZ_RS = 2048;   // rows per ahz split (z chunk in LDS, 32 KB)
constexpr int AHZ_CPW = 8;     // columns per ahz wave
constexpr int AHZ_COLS = 4 * AHZ_CPW;  // columns per ahz workgroup
constexpr int PX_JC = 256;     // columns per workgroup of the P x partials
constexpr int RES_KMAX = 1024; // LDS holds u_J for k <= RES_KMAX

struct ResPlan {
  int64_t nb_ax;   // ax row blocks
  int64_t S_z;     // ax column splits
  int64_t cpz;     // columns per ax split
  int64_t S_u;     // ahz row splits
  int64_t rpu;     // rows per ahz split
  int64_t nb_px;   // P x partial blocks
  int64_t nb_n;    // 256-blocks over n
  int64_t nb_m;    // 256-blocks over m
};

ResPlan plan_res(int64_t m, int64_t n) {
  ResPlan p;
  p.nb_ax = (m + AX_ROWS - 1) / AX_ROWS;
  int64_t S = (2048 + p.nb_ax - 1) / p.nb_ax;
  const int64_t maxS = (n + 31) / 32;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  p.cpz = (n + S - 1) / S;
  if (p.cpz < 1) p.cpz = 1;
  p.S_z = (n + p.cpz - 1) / p.cpz;
  if (p.S_z < 1) p.S_z = 1;
  p.rpu = AHZ_RS;
  p.S_u = (m + p.rpu - 1) / p.rpu;
  if (p.S_u < 1) p.S_u = 1;
  p.nb_px = (n + PX_JC - 1) / PX_JC;
  p.nb_n = (n + 255) / 256;
  p.nb_m = (m + 255) / 256;
  return p;
}

struct ResWs {
  double2 *x, *xth, *xtl, *z, *uh, *ul;
  double *pxpart, *zpart, *upart, *zn_part, *wn_part, *scal;
};

template <class C>
ResWs carve_res(C &c, int64_t m, int64_t n, int64_t k, const ResPlan &p) {
  ResWs w;
  w.x = c.template take<double2>(n);
  w.xth = c.template take<double2>(n);
  w.xtl = c.template take<double2>(n);
  w.z = c.template take<double2>(m);
  w.uh = c.template take<double2>(n);
  w.ul = c.template take<double2>(n);
  w.pxpart = c.template take<double>(size_t(p.nb_px) * size_t(k > 0 ? k : 1) * 4);
  w.zpart = c.template take<double>(size_t(p.S_z) * size_t(m) * 4);
  w.upart = c.template take<double>(size_t(p.S_u) * size_t(n) * 4);
  w.zn_part = c.template take<double>(p.nb_m);
  w.wn_part = c.template take<double>(p.nb_n);
  w.scal = c.template take<double>(4);
  return w;
}

// scal[0] = last sigma, scal[1] = stopped flag, scal[2] = norm divisor
RID_DEV bool stopped(const double *scal) { return scal[1] != 0.0; }

// Sum v over a 256-thread block in a fixed order; result in thread 0.
RID_DEV double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

__global__ __launch_bounds__(256) void x0_kernel(int64_t n, uint64_t seed, double2 *x,
                                                 double *parts, double *scal) {
  __shared__ double sh[4];
  const int64_t j = blockIdx.x * int64_t(256) + threadIdx.x;
  double v = 0.0;
  if (j < n) {
    const double2 g = rid_gauss(seed, 1u, 0u, static_cast<uint64_t>(j));
    x[j] = g;
    v = g.x * g.x + g.y * g.y;
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[0] = 0.0;
    scal[1] = 0.0;
  }
}

// Norm of a vector from its block partial sums; sets the stop flag when zero.
__global__ __launch_bounds__(256) void wnorm_final_kernel(int64_t nparts, const double *parts,
                                                          double *scal) {
  __shared__ double sh[4];
  if (stopped(scal)) return;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) v += parts[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(s);
    if (nrm == 0.0)
      scal[1] = 1.0;
    else
      scal[2] = nrm;
  }
}

__global__ __launch_bounds__(256) void x_scale_kernel(int64_t n, double2 *x,
                                                      const double *scal) {
  if (stopped(scal)) return;
  const int64_t j = blockIdx.x * int64_t(256) + threadIdx.x;
  if (j < n) {
    const double d = scal[2];
    x[j] = make_double2(x[j].x / d, x[j].y / d);
  }
}

__global__ __launch_bounds__(256) void xt_init_kernel(int64_t n, const double2 *x, double2 *xth,
                                                      double2 *xtl, const double *scal) {
  if (stopped(scal)) return;
  const int64_t j = blockIdx.x * int64_t(256) + threadIdx.x;
  if (j < n) {
    xth[j] = x[j];
    xtl[j] = make_double2(0.0, 0.0);
  }
}

// partial (P x)_t over the column block, compensated
__global__ __launch_bounds__(256) void px_partial_kernel(int64_t n, int64_t k,
                                                         const double2 *__restrict__ P,
                                                         int64_t ldp,
                                                         const double2 *__restrict__ x,
                                                         double *pxpart, const double *scal) {
  if (stopped(scal)) return;
  const int64_t j0 = int64_t(blockIdx.x) * PX_JC;
  const int64_t j1 = min(n, j0 + PX_JC);
  for (int64_t t = threadIdx.x; t < k; t += 256) {
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
      const double2 pe = P[t + j * ldp];
      const double2 xj = x[j];
      dot2_acc(sr, cr, pe.x, xj.x);
      dot2_acc(sr, cr, -pe.y, xj.y);
      dot2_acc(si, ci, pe.x, xj.y);
      dot2_acc(si, ci, pe.y, xj.x);
    }
    double *o = pxpart + (int64_t(blockIdx.x) * k + t) * 4;
    o[0] = sr;
    o[1] = cr;
    o[2] = si;
    o[3] = ci;
  }
}

// x~_{J[t]} = x_{J[t]} - (P x)_t as a double-double pair
__global__ __launch_bounds__(256) void px_final_kernel(int64_t n, int64_t k, int64_t nparts,
                                                       const int64_t *J, const double2 *x,
                                                       const double *pxpart, double2 *xth,
                                                       double2 *xtl, const double *scal) {
  if (stopped(scal)) return;
  const int64_t t = blockIdx.x * int64_t(256) + threadIdx.x;
  if (t >= k) return;
  double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
  for (int64_t b = 0; b < nparts; ++b) {
    const double *o = pxpart + (b * k + t) * 4;
    dd_add(sr, cr, o[0], o[1]);
    dd_add(si, ci, o[2], o[3]);
  }
  const int64_t jt = J[t];
  if (jt < 0 || jt >= n) return;
  const double2 xj = x[jt];
  double ar = xj.x, ac = 0.0, ai = xj.y, aci = 0.0;
  dd_add(ar, ac, -sr, -cr);
  dd_add(ai, aci, -si, -ci);
  double hr, lr, hi, li;
  dd_norm(ar, ac, hr, lr);
  dd_norm(ai, aci, hi, li);
  xth[jt] = make_double2(hr, hi);
  xtl[jt] = make_double2(lr, li);
}

// Two rows of A, widened to double, at column offset `off` (elements).  For
// complex128 the thread's rows are i0 and i0 + 256 (two 16-byte loads); for
// complex64 they are the adjacent rows i0, i0 + 1, read with one 16-byte
// load when the address is 16-byte aligned (PAIR) and with two 8-byte loads
// otherwise.
template <class TA, bool PAIR>
struct RowPair;
template <bool PAIR>
struct RowPair<double2, PAIR> {
  static constexpr int STEP = 256;  // distance between the thread's two rows
  static constexpr int LANE = 1;    // rows per thread index
  RID_DEV static void load(const double2 *p0, const double2 *p1, bool ok0, bool ok1,
                           int64_t off, double2 &a0, double2 &a1) {
    a0 = ok0 ? ld_stream(p0 + off) : make_double2(0.0, 0.0);
    a1 = ok1 ? ld_stream(p1 + off) : make_double2(0.0, 0.0);
  }
};
template <bool PAIR>
struct RowPair<float2, PAIR> {
  static constexpr int STEP = 1;
  static constexpr int LANE = 2;
  RID_DEV static void load(const float2 *p0, const float2 *p1, bool ok0, bool ok1, int64_t off,
                           double2 &a0, double2 &a1) {
    if (PAIR && ok1) {
      ld_stream_pair(p0 + off, a0, a1);
    } else {
      a0 = ok0 ? ld_stream(p0 + off) : make_double2(0.0, 0.0);
      a1 = ok1 ? ld_stream(p1 + off) : make_double2(0.0, 0.0);
    }
  }
};

// z partials: rows [512 rb, +512) x columns of split s.  TA is the storage
// type of A (complex128 or complex64, widened to double on load).
template <class TA, bool PAIR>
__global__ __launch_bounds__(256) void ax_partial_kernel(int64_t m, int64_t n,
                                                         const TA *__restrict__ A,
                                                         int64_t lda,
                                                         const double2 *__restrict__ xth,
                                                         const double2 *__restrict__ xtl,
                                                         int64_t cpz, double *zpart,
                                                         const double *scal) {
  using RP = RowPair<TA, PAIR>;
  if (stopped(scal)) return;
  const int64_t i0 = int64_t(blockIdx.x) * AX_ROWS + RP::LANE * threadIdx.x;
  const int64_t i1 = i0 + RP::STEP;
  const bool ok0 = i0 < m, ok1 = i1 < m;
  const int64_t jb = int64_t(blockIdx.y) * cpz;
  const int64_t je = min(n, jb + cpz);
  double s0r = 0, c0r = 0, s0i = 0, c0i = 0;
  double s1r = 0, c1r = 0, s1i = 0, c1i = 0;
  const TA *a0p = A + (ok0 ? i0 : 0);
  const TA *a1p = A + (ok1 ? i1 : 0);
  auto acc = [&](const double2 &a0, const double2 &a1, const double2 &xh, const double2 &xl) {
    dot2_acc(s0r, c0r, a0.x, xh.x);
    dot2_acc(s0r, c0r, -a0.y, xh.y);
    dot2_acc(s0i, c0i, a0.x, xh.y);
    dot2_acc(s0i, c0i, a0.y, xh.x);
    c0r = fma(a0.x, xl.x, c0r);
    c0r = fma(-a0.y, xl.y, c0r);
    c0i = fma(a0.x, xl.y, c0i);
    c0i = fma(a0.y, xl.x, c0i);
    dot2_acc(s1r, c1r, a1.x, xh.x);
    dot2_acc(s1r, c1r, -a1.y, xh.y);
    dot2_acc(s1i, c1i, a1.x, xh.y);
    dot2_acc(s1i, c1i, a1.y, xh.x);
    c1r = fma(a1.x, xl.x, c1r);
    c1r = fma(-a1.y, xl.y, c1r);
    c1i = fma(a1.x, xl.y, c1i);
    c1i = fma(a1.y, xl.x, c1i);
  };
  int64_t j = jb;
  for (; j + 4 <= je; j += 4) {
    double2 a0[4], a1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) RP::load(a0p, a1p, ok0, ok1, (j + u) * lda, a0[u], a1[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc(a0[u], a1[u], xth[j + u], xtl[j + u]);
  }
  for (; j < je; ++j) {
    double2 a0, a1;
    RP::load(a0p, a1p, ok0, ok1, j * lda, a0, a1);
    acc(a0, a1, xth[j], xtl[j]);
  }
  double *zp = zpart + int64_t(blockIdx.y) * m * 4;
  if (ok0) {
    zp[i0 * 4 + 0] = s0r;
    zp[i0 * 4 + 1] = c0r;
    zp[i0 * 4 + 2] = s0i;
    zp[i0 * 4 + 3] = c0i;
  }
  if (ok1) {
    zp[i1 * 4 + 0] = s1r;
    zp[i1 * 4 + 1] = c1r;
    zp[i1 * 4 + 2] = s1i;
    zp[i1 * 4 + 3] = c1i;
  }
}

__global__ __launch_bounds__(256) void z_final_kernel(int64_t m, int64_t S, const double *zpart,
                                                      double2 *z, double *parts,
                                                      const double *scal) {
  __shared__ double sh[4];
  if (stopped(scal)) return;
  const int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
  double v = 0.0;
  if (i < m) {
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (int64_t s = 0; s < S; ++s) {
      const double *o = zpart + (s * m + i) * 4;
      dd_add(sr, cr, o[0], o[1]);
      dd_add(si, ci, o[2], o[3]);
    }
    const double zr = sr + cr, zi = si + ci;
    z[i] = make_double2(zr, zi);
    v = zr * zr + zi * zi;
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sigma_final_kernel(int64_t nparts, const double *parts,
                                                          double *scal, double *sigma,
                                                          double *hist, int t) {
  __shared__ double sh[4];
  if (stopped(scal)) {
    if (threadIdx.x == 0 && hist) hist[t] = scal[0];
    return;
  }
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) v += parts[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const double sg = sqrt(s);
    scal[0] = sg;
    *sigma = sg;
    if (hist) hist[t] = sg;
  }
}

// u partials: columns [32 cb, +32) x rows of split s; z chunk staged in LDS.
// A lane takes one row per step for complex128 and two adjacent rows (one
// 16-byte load when aligned) for complex64.
template <class TA, bool PAIR>
__global__ __launch_bounds__(256) void ahz_partial_kernel(int64_t m, int64_t n,
                                                          const TA *__restrict__ A,
                                                          int64_t lda,
                                                          const double2 *__restrict__ z,
                                                          int64_t rpu, double *upart,
                                                          const double *scal) {
  constexpr bool C64 = sizeof(TA) == 8;
  __shared__ double2 zs[AHZ_RS];
  if (stopped(scal)) return;
  const int64_t r0 = int64_t(blockIdx.y) * rpu;
  const int64_t r1 = min(m, r0 + rpu);
  const int rows = static_cast<int>(r1 - r0);
  for (int i = threadIdx.x; i < rows; i += 256) zs[i] = z[r0 + i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t jb = int64_t(blockIdx.x) * AHZ_COLS + wave * AHZ_CPW;
  double sr[AHZ_CPW], cr[AHZ_CPW], si[AHZ_CPW], ci[AHZ_CPW];
  const TA *cp[AHZ_CPW];
  bool cok[AHZ_CPW];
#pragma unroll
  for (int u = 0; u < AHZ_CPW; ++u) {
    sr[u] = cr[u] = si[u] = ci[u] = 0.0;
    cok[u] = (jb + u) < n;
    cp[u] = A + (cok[u] ? (jb + u) : 0) * lda + r0;
  }
  auto acc = [&](int u, const double2 &a, const double2 &zz) {
    // conj(a) z = (ar zr + ai zi) + i (ar zi - ai zr)
    dot2_acc(sr[u], cr[u], a.x, zz.x);
    dot2_acc(sr[u], cr[u], a.y, zz.y);
    dot2_acc(si[u], ci[u], a.x, zz.y);
    dot2_acc(si[u], ci[u], -a.y, zz.x);
  };
  if (!C64) {
    for (int i = lane; i < rows; i += 64) {
      const double2 zz = zs[i];
      double2 a[AHZ_CPW];
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u)
        a[u] = cok[u] ? ld_stream(cp[u] + i) : make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u) acc(u, a[u], zz);
    }
  } else {
    for (int i = 2 * lane; i < rows; i += 128) {
      const bool two = i + 1 < rows;
      const double2 z0 = zs[i];
      const double2 z1 = two ? zs[i + 1] : make_double2(0.0, 0.0);
      double2 a0[AHZ_CPW], a1[AHZ_CPW];
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u) {
        if (!cok[u]) {
          a0[u] = a1[u] = make_double2(0.0, 0.0);
        } else if (PAIR && two) {
          ld_stream_pair(reinterpret_cast<const float2 *>(cp[u]) + i, a0[u], a1[u]);
        } else {
          a0[u] = ld_stream(cp[u] + i);
          a1[u] = two ? ld_stream(cp[u] + i + 1) : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u) {
        acc(u, a0[u], z0);
        acc(u, a1[u], z1);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < AHZ_CPW; ++u) {
    wave_sum_dd(sr[u], cr[u]);
    wave_sum_dd(si[u], ci[u]);
    if (lane == 0 && cok[u]) {
      double *o = upart + (int64_t(blockIdx.y) * n + jb + u) * 4;
      o[0] = sr[u];
      o[1] = cr[u];
      o[2] = si[u];
      o[3] = ci[u];
    }
  }
}

__global__ __launch_bounds__(256) void u_final_kernel(int64_t n, int64_t S, const double *upart,
                                                      double2 *uh, double2 *ul,
                                                      const double *scal) {
  if (stopped(scal)) return;
  const int64_t j = blockIdx.x * int64_t(256) + threadIdx.x;
  if (j >= n) return;
  double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
  for (int64_t s = 0; s < S; ++s) {
    const double *o = upart + (s * n + j) * 4;
    dd_add(sr, cr, o[0], o[1]);
    dd_add(si, ci, o[2], o[3]);
  }
  double hr, lr, hi, li;
  dd_norm(sr, cr, hr, lr);
  dd_norm(si, ci, hi, li);
  uh[j] = make_double2(hr, hi);
  ul[j] = make_double2(lr, li);
}

// w_j = u_j - sum_t conj(P(t, j)) u_{J[t]}, compensated; x <- w (unscaled)
__global__ __launch_bounds__(256) void w_kernel(int64_t n, int64_t k,
                                                const double2 *__restrict__ P, int64_t ldp,
                                                const int64_t *__restrict__ J,
                                                const double2 *__restrict__ uh,
                                                const double2 *__restrict__ ul, double2 *x,
                                                double *parts, const double *scal) {
  __shared__ double2 ujh[RES_KMAX];
  __shared__ double2 ujl[RES_KMAX];
  __shared__ double sh[4];
  if (stopped(scal)) return;
  for (int64_t t = threadIdx.x; t < k; t += 256) {
    const int64_t jt = J[t];
    const bool ok = jt >= 0 && jt < n;
    ujh[t] = ok ? uh[jt] : make_double2(0.0, 0.0);
    ujl[t] = ok ? ul[jt] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int64_t j = blockIdx.x * int64_t(256) + threadIdx.x;
  double v = 0.0;
  if (j < n) {
    const double2 h = uh[j], lo = ul[j];
    double sr = h.x, cr = lo.x, si = h.y, ci = lo.y;
    const double2 *pc = P + j * ldp;
    for (int64_t t = 0; t < k; ++t) {
      const double2 pe = pc[t];
      const double2 a = ujh[t], b = ujl[t];
      // conj(p) u = (pr ur + pi ui) + i (pr ui - pi ur)
      dot2_acc(sr, cr, -pe.x, a.x);
      dot2_acc(sr, cr, -pe.y, a.y);
      cr = fma(-pe.x, b.x, cr);
      cr = fma(-pe.y, b.y, cr);
      dot2_acc(si, ci, -pe.x, a.y);
      dot2_acc(si, ci, pe.y, a.x);
      ci = fma(-pe.x, b.y, ci);
      ci = fma(pe.y, b.x, ci);
    }
    const double wr = sr + cr, wi = si + ci;
    x[j] = make_double2(wr, wi);
    v = wr * wr + wi * wi;
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

}  // namespace

size_t residual_ws_bytes(int64_t m, int64_t n, int64_t k, int q) {
  (void)q;
  const ResPlan p = plan_res(m, n);
  WsCarve c(nullptr);
  carve_res(c, m, n, k, p);
  return c.off + 256;
}

template <class TA, bool PAIR>
hipError_t residual_impl(hipStream_t st, int64_t m, int64_t n, int64_t k, const TA *A,
                         int64_t lda, const int64_t *J, const double2 *P, int64_t ldp, int q,
                         uint64_t seed, double *sigma, double *hist, void *ws, RidProf *prof) {
  if (k > RES_KMAX) return hipErrorInvalidValue;
  const ResPlan p = plan_res(m, n);
  WsCarve c(ws);
  const ResWs w = carve_res(c, m, n, k, p);
  const dim3 blk(256);
  const dim3 gn(static_cast<unsigned>(p.nb_n));
  const dim3 gm(static_cast<unsigned>(p.nb_m));
  hipLaunchKernelGGL(x0_kernel, gn, blk, 0, st, n, seed, w.x, w.wn_part, w.scal);
  hipLaunchKernelGGL(wnorm_final_kernel, dim3(1), blk, 0, st, p.nb_n, w.wn_part, w.scal);
  hipLaunchKernelGGL(x_scale_kernel, gn, blk, 0, st, n, w.x, w.scal);
  for (int t = 0; t < q; ++t) {
    hipLaunchKernelGGL(xt_init_kernel, gn, blk, 0, st, n, w.x, w.xth, w.xtl, w.scal);
    if (k > 0) {
      hipLaunchKernelGGL(px_partial_kernel, dim3(static_cast<unsigned>(p.nb_px)), blk, 0, st,
                         n, k, P, ldp, w.x, w.pxpart, w.scal);
      hipLaunchKernelGGL(px_final_kernel, dim3(static_cast<unsigned>((k + 255) / 256)), blk, 0,
                         st, n, k, p.nb_px, J, w.x, w.pxpart, w.xth, w.xtl, w.scal);
    }
    {
      ProfScope ps(prof, st, RID_KERNEL_AX);
      hipLaunchKernelGGL((ax_partial_kernel<TA, PAIR>),
                         dim3(static_cast<unsigned>(p.nb_ax), static_cast<unsigned>(p.S_z)),
                         blk, 0, st, m, n, A, lda, w.xth, w.xtl, p.cpz, w.zpart, w.scal);
    }
    hipLaunchKernelGGL(z_final_kernel, gm, blk, 0, st, m, p.S_z, w.zpart, w.z, w.zn_part,
                       w.scal);
    hipLaunchKernelGGL(sigma_final_kernel, dim3(1), blk, 0, st, p.nb_m, w.zn_part, w.scal,
                       sigma, hist, t);
    if (t + 1 < q) {
      {
        ProfScope ps(prof, st, RID_KERNEL_AHZ);
        hipLaunchKernelGGL((ahz_partial_kernel<TA, PAIR>),
                           dim3(static_cast<unsigned>((n + AHZ_COLS - 1) / AHZ_COLS),
                                static_cast<unsigned>(p.S_u)),
                           blk, 0, st, m, n, A, lda, w.z, p.rpu, w.upart, w.scal);
      }
      hipLaunchKernelGGL(u_final_kernel, gn, blk, 0, st, n, p.S_u, w.upart, w.uh, w.ul,
                         w.scal);
      hipLaunchKernelGGL(w_kernel, gn, blk, 0, st, n, k, P, ldp, J, w.uh, w.ul, w.x,
                         w.wn_part, w.scal);
      hipLaunchKernelGGL(wnorm_final_kernel, dim3(1), blk, 0, st, p.nb_n, w.wn_part, w.scal);
      hipLaunchKernelGGL(x_scale_kernel, gn, blk, 0, st, n, w.x, w.scal);
    }
  }
  return hipGetLastError();
}

hipError_t launch_residual(hipStream_t st, rid_dtype dtype, int64_t m, int64_t n, int64_t k,
                           const void *A, int64_t lda, const int64_t *J, const double2 *P,
                           int64_t ldp, int q, uint64_t seed, double *sigma, double *hist,
                           void *ws, RidProf *prof) {
  if (dtype == RID_C64) {
    // pairs of adjacent entries are 16-byte aligned when A is and lda is even
    const bool pair = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    if (pair)
      return residual_impl<float2, true>(st, m, n, k, static_cast<const float2 *>(A), lda, J, P,
                                         ldp, q, seed, sigma, hist, ws, prof);
    return residual_impl<float2, false>(st, m, n, k, static_cast<const float2 *>(A), lda, J, P,
                                        ldp, q, seed, sigma, hist, ws, prof);
  }
  return residual_impl<double2, false>(st, m, n, k, static_cast<const double2 *>(A), lda, J, P,
                                       ldp, q, seed, sigma, hist, ws, prof);
}
