// residual.hip -- the error ||A - A(:,J) P||_2 of Table 5, estimated by power
// iteration on E = A - A(:,J) P without forming E:
//   E x   = A x~,           x~ = x - S_J (P x)       (S_J scatters to rows J)
//   E^H z = u - P^H u_J,    u  = A^H z
// E is ~1e-10 of A, so both products cancel almost completely.  Every sum
// over A is therefore compensated (Ogita-Rump-Oishi Dot2: exact products by
// FMA, TwoSum for the running sum, errors collected in a second double) and
// x~, u and the P-corrections are carried as double-double pairs.
//
// The two passes over A take one of three accumulations (RES_*, per job):
//   RES_DOT2  the compensated sums above (the double-precision ID);
//   RES_FP64  plain double FMA chains, x~ rounded to double: for the
//             reduced-precision forms, whose error is far above the
//             rounding of plain double sums (u sqrt(m + n) ||A||_F / sigma);
//   RES_FP32  single-precision products and sums within a workgroup's
//             slab, the partials combined in double (reported variant).
// The O(n k) side steps stay compensated in every mode.
//
// The two passes over A are the HBM-bound kernels of the whole ID; both read
// A with non-temporal loads (A is touched once per pass):
//   ax  : z = A x~ ; a workgroup streams a 512-row slab of a range of
//         columns (each column slab is one contiguous 8 KB read).
//   ahz : u = A^H z ; a workgroup stages a 2048-row chunk of z in LDS and
//         each wave streams AHZ_CPW columns of that chunk (32 KB contiguous
//         reads each for complex128), reducing in registers then across
//         lanes by one reduce-scatter.
// Partial sums over column splits (resp. row splits) are reduced in a fixed
// order by separate kernels, so results are bitwise reproducible.
//
// Every kernel body takes a per-job descriptor (ResJob) and a block index
// inside that job, so the same bodies serve one ID (one launch per step,
// grid = the job's blocks) and a batch of IDs (one launch per step over all
// jobs, each block looking up its (job, block) pair in a table).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "rid_internal.hpp"

namespace {

constexpr int AX_ROWS = 512;   // rows per ax workgroup (2 per thread)
constexpr int AHZ_RS = 2048;   // rows per ahz split (z chunk in LDS, 32 KB)
// columns per ahz wave: a plan choice, 8 (fewer z reads per byte of A) or 4
// (fewer registers: 5 waves per SIMD instead of 3 for complex64)

constexpr int PX_SETS = 1024;  // most column sets of the P x partials (one per wave)
constexpr int RES_KMAX = 1024; // largest k of the residual (as of the interpolation)

struct ResPlan {
  int64_t nb_ax;   // ax row blocks (ax_h rows each)
  int ax_h;        // rows per ax row block: 512, or 256 / 128 for the paired complex64
                   // body, whose workgroup then takes 512 / ax_h column splits
  int64_t nb_axy;  // ax grid y: column splits / (512 / ax_h), rounded up
  int64_t S_z;     // ax column splits
  int64_t cpz;     // columns per ax split
  int64_t S_u;     // ahz row splits
  int64_t rpu;     // rows per ahz split
  int64_t nb_ahz;  // ahz column blocks
  int ahz_cpw;     // ahz columns per wave (4 or 8)
  int64_t nb_px;   // P x partial sets (column sets of px_cpw columns, one per wave)
  int64_t px_cpw;  // columns per P x partial set
  int64_t nb_pxb;  // P x partial workgroups (four sets each)
  int64_t nb_k;    // workgroups of the P x final step (four rows of P each)
  int64_t nb_n;    // 256-blocks over n
  int64_t nb_w;    // 64-blocks over n (the w step; its norm partials)
  int64_t nb_m;    // 256-blocks over m
};

// target_blocks: workgroups wanted for the ax pass of this job alone
ResPlan plan_res(int64_t m, int64_t n, int64_t k, int64_t target_blocks, int ahz_cpw) {
  ResPlan p;
  p.ahz_cpw = ahz_cpw == 4 ? 4 : 8;
  p.nb_ax = (m + AX_ROWS - 1) / AX_ROWS;
  int64_t S = (target_blocks + p.nb_ax - 1) / p.nb_ax;
  const int64_t maxS = (n + 31) / 32;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  p.cpz = (n + S - 1) / S;
  if (p.cpz < 1) p.cpz = 1;
  if (rid_tl_short_blocks && p.cpz > RID_AX_COLS_MAX) p.cpz = RID_AX_COLS_MAX;
  if ((n + p.cpz - 1) / p.cpz > 65535) p.cpz = (n + 65534) / 65535;  // grid y
  p.S_z = (n + p.cpz - 1) / p.cpz;
  if (p.S_z < 1) p.S_z = 1;
  p.ax_h = AX_ROWS;
  p.nb_axy = p.S_z;
  p.rpu = AHZ_RS;
  p.S_u = (m + p.rpu - 1) / p.rpu;
  if (p.S_u < 1) p.S_u = 1;
  p.nb_ahz = (n + 4 * p.ahz_cpw - 1) / (4 * p.ahz_cpw);
  p.nb_px = std::min<int64_t>((n + 15) / 16, PX_SETS);
  if (p.nb_px < 1) p.nb_px = 1;
  p.px_cpw = (n + p.nb_px - 1) / p.nb_px;
  if (p.px_cpw < 1) p.px_cpw = 1;
  p.nb_px = (n + p.px_cpw - 1) / p.px_cpw;
  if (p.nb_px < 1) p.nb_px = 1;
  p.nb_pxb = (p.nb_px + 3) / 4;
  p.nb_k = (k + 3) / 4;
  p.nb_n = (n + 255) / 256;
  p.nb_w = (n + 63) / 64;
  p.nb_m = (m + 255) / 256;
  return p;
}

// Row blocks of h rows for the ax pass (h = 128, 256 or 512): the column
// splits stay as planned, a workgroup takes 512 / h of them, so a workgroup
// still covers about the same bytes of A.
void set_ax_rows(ResPlan &p, int64_t m, int h) {
  p.ax_h = h;
  p.nb_ax = (m + h - 1) / h;
  const int64_t g = AX_ROWS / h;
  p.nb_axy = (p.S_z + g - 1) / g;
}

// One power-iteration problem: sizes, inputs, plan and workspace.
struct ResJob {
  int64_t m, n, k, lda, ldp;
  int acc;   // accumulation of the passes over A (RES_DOT2, RES_FP64, RES_FP32)
  const void *A;
  const int64_t *J;
  const double2 *P;
  uint64_t seed;
  double *sigma, *hist;
  int pair;  // complex64 A: adjacent entries may be read as one 16-byte load
  int al16;  // complex64 A with a 16-byte aligned base (any lda)
  ResPlan pl;
  double2 *x, *xth, *xtl, *z, *uh, *ul;
  double *pxpart, *zpart, *upart, *zn_part, *wn_part, *scal;
};

template <class C>
void carve_res(C &c, ResJob &r) {
  const ResPlan &p = r.pl;
  const int64_t m = r.m, n = r.n, k = r.k;
  r.x = c.template take<double2>(n);
  r.xth = c.template take<double2>(n);
  r.xtl = c.template take<double2>(n);
  r.z = c.template take<double2>(m);
  r.uh = c.template take<double2>(n);
  r.ul = c.template take<double2>(n);
  r.pxpart = c.template take<double>(size_t(p.nb_px) * size_t(k > 0 ? k : 1) * 4);
  r.zpart = c.template take<double>(size_t(p.S_z) * size_t(m) * 4);
  r.upart = c.template take<double>(size_t(p.S_u) * size_t(n) * 4);
  r.zn_part = c.template take<double>(p.nb_m);
  r.wn_part = c.template take<double>(p.nb_w > 0 ? p.nb_w : 1);
  r.scal = c.template take<double>(4);
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

// ------------------------------------------------------------------ bodies
// The norm partials of x are per 64 columns (one per wave here, one per
// workgroup of the w step).
RID_DEV void x0_body(const ResJob &r, int64_t bx) {
  const int64_t j = bx * 256 + threadIdx.x;
  double v = 0.0;
  if (j < r.n) {
    const double2 g = rid_gauss(r.seed, 1u, 0u, static_cast<uint64_t>(j));
    r.x[j] = g;
    v = g.x * g.x + g.y * g.y;
  }
  v = wave_sum(v);
  const int64_t g64 = bx * 4 + (threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0 && g64 < r.pl.nb_w) r.wn_part[g64] = v;
  if (bx == 0 && threadIdx.x == 0) {
    r.scal[0] = 0.0;
    r.scal[1] = 0.0;
  }
}

// Norm of x from its block partial sums; sets the stop flag when zero.
RID_DEV void wnorm_final_body(const ResJob &r) {
  __shared__ double sh[4];
  if (stopped(r.scal)) return;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < r.pl.nb_w; i += 256) v += r.wn_part[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(s);
    if (nrm == 0.0)
      r.scal[1] = 1.0;
    else
      r.scal[2] = nrm;
  }
}

RID_DEV void x_scale_body(const ResJob &r, int64_t bx) {
  if (stopped(r.scal)) return;
  const int64_t j = bx * 256 + threadIdx.x;
  if (j < r.n) {
    const double d = r.scal[2];
    r.x[j] = make_double2(r.x[j].x / d, r.x[j].y / d);
  }
}

RID_DEV void xt_init_body(const ResJob &r, int64_t bx) {
  if (stopped(r.scal)) return;
  const int64_t j = bx * 256 + threadIdx.x;
  if (j < r.n) {
    r.xth[j] = r.x[j];
    r.xtl[j] = make_double2(0.0, 0.0);
  }
}

// partial (P x)_t over a block of columns, compensated
// (P x)_t over one column set, for every t: wave w of workgroup bx takes
// set 4 bx + w (columns px_cpw (4 bx + w) ..), its lanes rows t = lane + 64 h
// of those columns (coalesced reads of P), compensated sums in column order.
RID_DEV void px_partial_body(const ResJob &r, int64_t bx) {
  if (stopped(r.scal)) return;
  const int lane = threadIdx.x & 63;
  const int64_t set = bx * 4 + (threadIdx.x >> 6);
  if (set >= r.pl.nb_px) return;
  const int64_t j0 = set * r.pl.px_cpw;
  const int64_t j1 = min(r.n, j0 + r.pl.px_cpw);
  for (int64_t tb = 0; tb < r.k; tb += 64) {
    const int64_t t = tb + lane;
    const bool ok = t < r.k;
    const double2 *pc = r.P + (ok ? t : 0);
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    // unrolled so that several loads are in flight; the sums keep their order
#pragma unroll 8
    for (int64_t j = j0; j < j1; ++j) {
      const double2 pv = pc[j * r.ldp];
      const double2 pe = ok ? pv : make_double2(0.0, 0.0);
      const double2 xj = r.x[j];
      dot2_acc(sr, cr, pe.x, xj.x);
      dot2_acc(sr, cr, -pe.y, xj.y);
      dot2_acc(si, ci, pe.x, xj.y);
      dot2_acc(si, ci, pe.y, xj.x);
    }
    if (ok) {
      double *o = r.pxpart + (set * r.k + t) * 4;
      o[0] = sr;
      o[1] = cr;
      o[2] = si;
      o[3] = ci;
    }
  }
}

// x~_{J[t]} = x_{J[t]} - (P x)_t as a double-double pair: wave w of
// workgroup bx takes t = 4 bx + w, its lanes the partial sets lane,
// lane + 64, ..., and a compensated wave sum joins them.
RID_DEV void px_final_body(const ResJob &r, int64_t bx) {
  if (stopped(r.scal)) return;
  const int lane = threadIdx.x & 63;
  const int64_t t = bx * 4 + (threadIdx.x >> 6);
  if (t >= r.k) return;
  double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
  for (int64_t b = lane; b < r.pl.nb_px; b += 64) {
    const double *o = r.pxpart + (b * r.k + t) * 4;
    dd_add(sr, cr, o[0], o[1]);
    dd_add(si, ci, o[2], o[3]);
  }
  wave_sum_dd(sr, cr);
  wave_sum_dd(si, ci);
  if (lane != 0) return;
  const int64_t jt = r.J[t];
  if (jt < 0 || jt >= r.n) return;
  const double2 xj = r.x[jt];
  double ar = xj.x, ac = 0.0, ai = xj.y, aci = 0.0;
  dd_add(ar, ac, -sr, -cr);
  dd_add(ai, aci, -si, -ci);
  double hr, lr, hi, li;
  dd_norm(ar, ac, hr, lr);
  dd_norm(ai, aci, hi, li);
  r.xth[jt] = make_double2(hr, hi);
  r.xtl[jt] = make_double2(lr, li);
}

// Two rows of A, widened to double, at element offset `off`.  complex128:
// the thread's rows are i0 and i0 + 256 (two 16-byte loads); complex64: the
// adjacent rows i0, i0 + 1, one 16-byte load when the pair is 16-byte
// aligned, else two 8-byte loads.
template <class TA>
struct RowPair;
template <>
struct RowPair<double2> {
  static constexpr int STEP = 256;  // distance between the thread's two rows
  static constexpr int LANE = 1;    // rows per thread index
  // p0 and p1 point into A even for rows past m (the caller clamps them), so
  // both loads are issued unconditionally and the rows past m are zeroed
  RID_DEV static void load(const double2 *p0, const double2 *p1, bool ok0, bool ok1, int64_t off,
                           bool, double2 &a0, double2 &a1) {
    const double2 v0 = ld_stream(p0 + off), v1 = ld_stream(p1 + off);
    a0 = ok0 ? v0 : make_double2(0.0, 0.0);
    a1 = ok1 ? v1 : make_double2(0.0, 0.0);
  }
};
template <>
struct RowPair<float2> {
  static constexpr int STEP = 1;
  static constexpr int LANE = 2;
  RID_DEV static void load(const float2 *p0, const float2 *p1, bool ok0, bool ok1, int64_t off,
                           bool pair, double2 &a0, double2 &a1) {
    if (pair && ok1) {
      ld_stream_pair(p0 + off, a0, a1);
    } else {
      a0 = ok0 ? ld_stream(p0 + off) : make_double2(0.0, 0.0);
      a1 = ok1 ? ld_stream(p1 + off) : make_double2(0.0, 0.0);
    }
  }
};

// z partials: rows [512 bx, +512) x columns of split by
// WIDE: the fast path below (one ID's large slabs); the grouped kernels of a
// batch leave it out, as their small jobs rarely take it and would pay its
// registers
template <class TA, bool WIDE, int ACC>
RID_DEV void ax_body(const ResJob &r, int64_t bx, int64_t by) {
  using RP = RowPair<TA>;
  if (stopped(r.scal)) return;
  const TA *A = static_cast<const TA *>(r.A);
  const int64_t m = r.m, lda = r.lda;
  const int64_t i0 = bx * AX_ROWS + RP::LANE * threadIdx.x;
  const int64_t i1 = i0 + RP::STEP;
  const bool ok0 = i0 < m, ok1 = i1 < m;
  const int64_t jb = by * r.pl.cpz;
  const int64_t je = min(r.n, jb + r.pl.cpz);
  const bool pair = r.pair != 0;
  const double2 *__restrict__ xth = r.xth;
  const double2 *__restrict__ xtl = r.xtl;
  double s0r = 0, c0r = 0, s0i = 0, c0i = 0;
  double s1r = 0, c1r = 0, s1i = 0, c1i = 0;
  float f0r = 0.0f, f0i = 0.0f, f1r = 0.0f, f1i = 0.0f;
  const TA *a0p = A + (ok0 ? i0 : 0);
  const TA *a1p = A + (ok1 ? i1 : 0);
  // x~ = xh + xl; xl is zero except on the k skeleton columns, so the xl
  // products (which only add to the compensation) are skipped for a group of
  // columns whose xl are all zero -- a uniform test, no divergence.  The
  // plain modes round x~ to xh and never read xl.
  auto acc_hi = [&](const double2 &a0, const double2 &a1, const double2 &xh) {
    if constexpr (ACC == RES_DOT2) {
      dot2_acc(s0r, c0r, a0.x, xh.x);
      dot2_acc(s0r, c0r, -a0.y, xh.y);
      dot2_acc(s0i, c0i, a0.x, xh.y);
      dot2_acc(s0i, c0i, a0.y, xh.x);
      dot2_acc(s1r, c1r, a1.x, xh.x);
      dot2_acc(s1r, c1r, -a1.y, xh.y);
      dot2_acc(s1i, c1i, a1.x, xh.y);
      dot2_acc(s1i, c1i, a1.y, xh.x);
    } else if constexpr (ACC == RES_FP64) {
      s0r = fma(a0.x, xh.x, s0r);
      s0r = fma(-a0.y, xh.y, s0r);
      s0i = fma(a0.x, xh.y, s0i);
      s0i = fma(a0.y, xh.x, s0i);
      s1r = fma(a1.x, xh.x, s1r);
      s1r = fma(-a1.y, xh.y, s1r);
      s1i = fma(a1.x, xh.y, s1i);
      s1i = fma(a1.y, xh.x, s1i);
    } else {
      const float xr = static_cast<float>(xh.x), xi = static_cast<float>(xh.y);
      const float a0r = static_cast<float>(a0.x), a0i = static_cast<float>(a0.y);
      const float a1r = static_cast<float>(a1.x), a1i = static_cast<float>(a1.y);
      f0r = fmaf(a0r, xr, f0r);
      f0r = fmaf(-a0i, xi, f0r);
      f0i = fmaf(a0r, xi, f0i);
      f0i = fmaf(a0i, xr, f0i);
      f1r = fmaf(a1r, xr, f1r);
      f1r = fmaf(-a1i, xi, f1r);
      f1i = fmaf(a1r, xi, f1i);
      f1i = fmaf(a1i, xr, f1i);
    }
  };
  auto acc_lo = [&](const double2 &a0, const double2 &a1, const double2 &xl) {
    if constexpr (ACC != RES_DOT2) return;
    c0r = fma(a0.x, xl.x, c0r);
    c0r = fma(-a0.y, xl.y, c0r);
    c0i = fma(a0.x, xl.y, c0i);
    c0i = fma(a0.y, xl.x, c0i);
    c1r = fma(a1.x, xl.x, c1r);
    c1r = fma(-a1.y, xl.y, c1r);
    c1i = fma(a1.x, xl.y, c1i);
    c1i = fma(a1.y, xl.x, c1i);
  };
  int64_t j = jb;
  if constexpr (WIDE) {
    // the whole slab inside A and, for complex64, 16-byte pairs allowed (a
    // uniform test): every load is unconditional (one pair load per thread
    // and column for complex64), and 8 columns are in flight at a time.  The
    // products and their order are those of the general loop below; only the
    // skeleton columns' low-word terms join the error sums in groups of 8
    // instead of 4.
    if ((sizeof(TA) == 16 || pair) && (bx + 1) * AX_ROWS <= m) {
      for (; j + 8 <= je; j += 8) {
        double2 a0[8], a1[8], xl[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if constexpr (sizeof(TA) == 8)
            ld_stream_pair(a0p + (j + u) * lda, a0[u], a1[u]);
          else
            RP::load(a0p, a1p, true, true, (j + u) * lda, pair, a0[u], a1[u]);
        }
        bool lo = false;
        if constexpr (ACC == RES_DOT2) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            xl[u] = ld_uniform(xtl, j + u);
            lo = lo || xl[u].x != 0.0 || xl[u].y != 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc_hi(a0[u], a1[u], ld_uniform(xth, j + u));
        if (lo) {
#pragma unroll
          for (int u = 0; u < 8; ++u) acc_lo(a0[u], a1[u], xl[u]);
        }
      }
    }
  }
  for (; j + 4 <= je; j += 4) {
    double2 a0[4], a1[4], xl[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) RP::load(a0p, a1p, ok0, ok1, (j + u) * lda, pair, a0[u], a1[u]);
    bool lo = false;
    if constexpr (ACC == RES_DOT2) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xl[u] = ld_uniform(xtl, j + u);
        lo = lo || xl[u].x != 0.0 || xl[u].y != 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc_hi(a0[u], a1[u], ld_uniform(xth, j + u));
    if (lo) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc_lo(a0[u], a1[u], xl[u]);
    }
  }
  for (; j < je; ++j) {
    double2 a0, a1;
    RP::load(a0p, a1p, ok0, ok1, j * lda, pair, a0, a1);
    acc_hi(a0, a1, ld_uniform(xth, j));
    if constexpr (ACC == RES_DOT2) acc_lo(a0, a1, ld_uniform(xtl, j));
  }
  if constexpr (ACC == RES_FP32) {
    s0r = f0r;
    s0i = f0i;
    s1r = f1r;
    s1i = f1i;
  }
  double *zp = r.zpart + by * m * 4;
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

// z partials for complex64 A with a 16-byte aligned base and plain sums:
// every entry arrives in a 16-byte load of two adjacent rows, whatever the
// parity of lda.  Column j starts on a 16-byte boundary when j lda is even
// (slab starts are even rows); there the thread's rows (i0, i0 + 1) are one
// pair, and their sums go to the first and third words of the rows' partial
// entries.  When j lda is odd (lda odd, j odd) the aligned pairs are
// (i0 - 1, i0): their sums go to the second and fourth words (unused by
// plain sums otherwise), so the slab's rows shifted by one are summed
// without any exchange between threads -- row 512 bx - 1 by this slab's
// thread 0, the row before it by the previous slab.  The z reduction adds
// all four words.  Every thread makes one 16-byte load per column.  Rows
// past m are loaded from 16-byte granules that hold a row of the column (so
// never from an unmapped page) and zeroed.  Row blocks are ax_h rows: 512
// (the general layout), or 256 / 128 for a short or ragged m, where the
// workgroup's thread groups take separate column splits.  With lda odd this
// needs m % ax_h != 0 (so that the last block's thread reaches row m - 1);
// the caller takes the general loop otherwise.
//
// Compensated sums (RES_DOT2) use all four words for the rows' sums and
// their errors, so they take this body for an even lda only (every column
// unshifted); the low words of x~ join the error sums as in the general
// loop.
template <int ACC, bool SX>
RID_DEV void ax_c64_paired(const ResJob &r, int64_t bx, int64_t by) {
  using Acc = typename std::conditional<ACC == RES_FP32, float, double>::type;
  // no early test of the stop flag: a stopped job's partials are computed
  // but never read (the z reduction tests it), and the A loads start sooner
  const float2 *A = static_cast<const float2 *>(r.A);
  const int64_t m = r.m, lda = r.lda;
  const int t = threadIdx.x;
  // the workgroup's threads form 512 / h groups of h / 2 threads; group g
  // takes rows [h bx, h bx + h) of column split by (512 / h) + g
  const int h = r.pl.ax_h;
  const int half = h >> 1;
  const int tg = t % half;
  // the same in every lane of a wave (a group is at least one wave): read
  // as uniform, so that the column loop's x~ loads are scalar loads
  const int64_t split = uniform_i64(by * (AX_ROWS / h) + t / half);
  const int64_t i0 = bx * h + 2 * tg;
  const bool ok0 = i0 < m, ok1 = i0 + 1 < m;
  const bool okm = i0 >= 1 && i0 - 1 < m;  // row i0 - 1 of a shifted pair
  const bool odd = (lda & 1) != 0;
  // a wave whose rows (shifted ones included) all lie past m, or whose
  // split lies past the last one, has no loads
  const bool live = __builtin_amdgcn_readfirstlane(
                        (bx * h + 128 * (tg >> 6) - 1 < m && split < r.pl.S_z) ? 1 : 0) != 0;
  // pair starts: unshifted (i0, or row 0 past m); shifted (i0 - 1, or row
  // -1 past m: the previous column's last stored entry, as j >= 1 there)
  const int64_t pu = ok0 ? i0 : 0;
  const int64_t ps = (i0 - 1 < m) ? i0 - 1 : -1;
  const int64_t jb = split * r.pl.cpz;
  const int64_t je = live ? min(r.n, jb + r.pl.cpz) : jb;
  const double2 *__restrict__ xth = r.xth;
  // x~ of a column, the same in every lane: a scalar load (SX, the batch's
  // passes: one scalar load per two columns instead of a vector load each)
  // or a plain load (one ID: the scalar form costs it a wave per SIMD)
  auto xload = [](const double2 *p, int64_t i) -> double2 {
    if constexpr (SX)
      return ld_uniform(p, i);
    else
      return p[i];
  };
  Acc s0r = 0, s0i = 0, s1r = 0, s1i = 0;  // rows i0, i0 + 1 (unshifted columns)
  Acc smr = 0, smi = 0, snr = 0, sni = 0;  // rows i0 - 1, i0 (shifted columns)
  const double2 zero2 = make_double2(0.0, 0.0);
  // a x for one entry into (sr, si); x~ is rounded to its high word
  auto fma_c = [&](Acc &sr, Acc &si, const double2 &a, const double2 &xh) {
    if constexpr (ACC != RES_FP32) {
      sr = fma(a.x, xh.x, sr);
      sr = fma(-a.y, xh.y, sr);
      si = fma(a.x, xh.y, si);
      si = fma(a.y, xh.x, si);
    } else {
      const float ar = static_cast<float>(a.x), ai = static_cast<float>(a.y);
      const float xr = static_cast<float>(xh.x), xi = static_cast<float>(xh.y);
      sr = fmaf(ar, xr, sr);
      sr = fmaf(-ai, xi, sr);
      si = fmaf(ar, xi, si);
      si = fmaf(ai, xr, si);
    }
  };
  if constexpr (ACC == RES_DOT2) {
    // lda even: one pair (i0, i0 + 1) per column; Dot2 sums of a x~_hi,
    // plain sums of a x~_lo into the errors where x~_lo is non-zero
    double c0r = 0, c0i = 0, c1r = 0, c1i = 0;
    const double2 *__restrict__ xtl = r.xtl;
    auto hi = [&](const double2 &a0, const double2 &a1, const double2 &xh) {
      const double2 p0 = ok0 ? a0 : zero2, p1 = ok1 ? a1 : zero2;
      dot2_acc(s0r, c0r, p0.x, xh.x);
      dot2_acc(s0r, c0r, -p0.y, xh.y);
      dot2_acc(s0i, c0i, p0.x, xh.y);
      dot2_acc(s0i, c0i, p0.y, xh.x);
      dot2_acc(s1r, c1r, p1.x, xh.x);
      dot2_acc(s1r, c1r, -p1.y, xh.y);
      dot2_acc(s1i, c1i, p1.x, xh.y);
      dot2_acc(s1i, c1i, p1.y, xh.x);
    };
    auto lo = [&](const double2 &a0, const double2 &a1, const double2 &xl) {
      const double2 p0 = ok0 ? a0 : zero2, p1 = ok1 ? a1 : zero2;
      c0r = fma(p0.x, xl.x, c0r);
      c0r = fma(-p0.y, xl.y, c0r);
      c0i = fma(p0.x, xl.y, c0i);
      c0i = fma(p0.y, xl.x, c0i);
      c1r = fma(p1.x, xl.x, c1r);
      c1r = fma(-p1.y, xl.y, c1r);
      c1i = fma(p1.x, xl.y, c1i);
      c1i = fma(p1.y, xl.x, c1i);
    };
    int64_t j = jb;
    for (; j + 8 <= je; j += 8) {
      double2 a0[8], a1[8], xl[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ld_stream_pair(A + (j + u) * lda + pu, a0[u], a1[u]);
      bool any = false;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        xl[u] = xload(xtl, j + u);
        any = any || xl[u].x != 0.0 || xl[u].y != 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) hi(a0[u], a1[u], xload(xth, j + u));
      if (any) {
#pragma unroll
        for (int u = 0; u < 8; ++u) lo(a0[u], a1[u], xl[u]);
      }
    }
    for (; j < je; ++j) {
      double2 a0, a1;
      ld_stream_pair(A + j * lda + pu, a0, a1);
      hi(a0, a1, xload(xth, j));
      lo(a0, a1, xload(xtl, j));
    }
    if (split >= r.pl.S_z) return;
    double *zp = r.zpart + split * m * 4;
    if (ok0) {
      zp[i0 * 4 + 0] = s0r;
      zp[i0 * 4 + 1] = c0r;
      zp[i0 * 4 + 2] = s0i;
      zp[i0 * 4 + 3] = c0i;
    }
    if (ok1) {
      zp[(i0 + 1) * 4 + 0] = s1r;
      zp[(i0 + 1) * 4 + 1] = c1r;
      zp[(i0 + 1) * 4 + 2] = s1i;
      zp[(i0 + 1) * 4 + 3] = c1i;
    }
    return;
  }
  auto unshifted = [&](const double2 &a0, const double2 &a1, const double2 &xh) {
    fma_c(s0r, s0i, ok0 ? a0 : zero2, xh);
    fma_c(s1r, s1i, ok1 ? a1 : zero2, xh);
  };
  auto shifted = [&](const double2 &b0, const double2 &b1, const double2 &xh) {
    fma_c(smr, smi, okm ? b0 : zero2, xh);
    fma_c(snr, sni, ok0 ? b1 : zero2, xh);
  };
  int64_t j = jb;
  if (odd) {
    // j lda odd exactly for odd j: a group of 8 from an even column holds
    // four unshifted (even u) and four shifted (odd u) columns
    if ((j & 1) && j < je) {
      double2 b0, b1;
      ld_stream_pair(A + j * lda + ps, b0, b1);
      shifted(b0, b1, xload(xth, j));
      ++j;
    }
    for (; j + 8 <= je; j += 8) {
      double2 a0[8], a1[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ld_stream_pair(A + (j + u) * lda + ((u & 1) ? ps : pu), a0[u], a1[u]);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (u & 1)
          shifted(a0[u], a1[u], xload(xth, j + u));
        else
          unshifted(a0[u], a1[u], xload(xth, j + u));
      }
    }
    for (; j < je; ++j) {
      double2 a0, a1;
      const bool sh = (j & 1) != 0;
      ld_stream_pair(A + j * lda + (sh ? ps : pu), a0, a1);
      if (sh)
        shifted(a0, a1, xload(xth, j));
      else
        unshifted(a0, a1, xload(xth, j));
    }
  } else {
    for (; j + 8 <= je; j += 8) {
      double2 a0[8], a1[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ld_stream_pair(A + (j + u) * lda + pu, a0[u], a1[u]);
#pragma unroll
      for (int u = 0; u < 8; ++u) unshifted(a0[u], a1[u], xload(xth, j + u));
    }
    for (; j < je; ++j) {
      double2 a0, a1;
      ld_stream_pair(A + j * lda + pu, a0, a1);
      unshifted(a0, a1, xload(xth, j));
    }
  }
  // words 0 and 2 of rows i0, i0 + 1; words 1 and 3 of rows i0 - 1, i0
  // (zero for lda even)
  if (split >= r.pl.S_z) return;
  double *zp = r.zpart + split * m * 4;
  if (ok0) {
    zp[i0 * 4 + 0] = static_cast<double>(s0r);
    zp[i0 * 4 + 1] = static_cast<double>(snr);
    zp[i0 * 4 + 2] = static_cast<double>(s0i);
    zp[i0 * 4 + 3] = static_cast<double>(sni);
  }
  if (ok1) {
    zp[(i0 + 1) * 4 + 0] = static_cast<double>(s1r);
    zp[(i0 + 1) * 4 + 2] = static_cast<double>(s1i);
    if (!odd) {
      zp[(i0 + 1) * 4 + 1] = 0.0;
      zp[(i0 + 1) * 4 + 3] = 0.0;
    }
  }
  if (odd && okm) {
    zp[(i0 - 1) * 4 + 1] = static_cast<double>(smr);
    zp[(i0 - 1) * 4 + 3] = static_cast<double>(smi);
  }
}

RID_DEV void z_final_body(const ResJob &r, int64_t bx) {
  __shared__ double sh[4];
  if (stopped(r.scal)) return;
  const int64_t i = bx * 256 + threadIdx.x;
  double v = 0.0;
  if (i < r.m) {
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    // unrolled so that several loads are in flight; the sums keep their order
#pragma unroll 8
    for (int64_t s = 0; s < r.pl.S_z; ++s) {
      const double *o = r.zpart + (s * r.m + i) * 4;
      dd_add(sr, cr, o[0], o[1]);
      dd_add(si, ci, o[2], o[3]);
    }
    const double zr = sr + cr, zi = si + ci;
    r.z[i] = make_double2(zr, zi);
    v = zr * zr + zi * zi;
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) r.zn_part[bx] = s;
}

RID_DEV void sigma_final_body(const ResJob &r, int t) {
  __shared__ double sh[4];
  if (stopped(r.scal)) {
    if (threadIdx.x == 0 && r.hist) r.hist[t] = r.scal[0];
    return;
  }
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < r.pl.nb_m; i += 256) v += r.zn_part[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const double sg = sqrt(s);
    r.scal[0] = sg;
    *r.sigma = sg;
    if (r.hist) r.hist[t] = sg;
  }
}

// u partials: columns [32 bx, +32) x rows of split by; z chunk staged in LDS.
// A lane takes one row per step for complex128 and two adjacent rows (one
// 16-byte load when aligned) for complex64.
template <class TA, int AHZ_CPW, int ACC>
RID_DEV void ahz_body(const ResJob &r, int64_t bx, int64_t by) {
  constexpr int AHZ_COLS = 4 * AHZ_CPW;  // columns per workgroup
  constexpr bool C64 = sizeof(TA) == 8;
  __shared__ double2 zs[AHZ_RS];
  if (stopped(r.scal)) return;
  const TA *A = static_cast<const TA *>(r.A);
  const int64_t m = r.m, n = r.n, lda = r.lda;
  const bool pair = r.pair != 0;
  const int64_t r0 = by * r.pl.rpu;
  const int64_t r1 = min(m, r0 + r.pl.rpu);
  const int rows = static_cast<int>(r1 - r0);
  for (int i = threadIdx.x; i < rows; i += 256) zs[i] = r.z[r0 + i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t jb = bx * AHZ_COLS + wave * AHZ_CPW;
  double sr[AHZ_CPW], cr[AHZ_CPW], si[AHZ_CPW], ci[AHZ_CPW];
  float fr[AHZ_CPW], fi[AHZ_CPW];
  const TA *cp[AHZ_CPW];
  bool cok[AHZ_CPW];
#pragma unroll
  for (int u = 0; u < AHZ_CPW; ++u) {
    sr[u] = cr[u] = si[u] = ci[u] = 0.0;
    fr[u] = fi[u] = 0.0f;
    cok[u] = (jb + u) < n;
    cp[u] = A + (cok[u] ? (jb + u) : 0) * lda + r0;
  }
  auto acc = [&](int u, const double2 &a, const double2 &zz) {
    // conj(a) z = (ar zr + ai zi) + i (ar zi - ai zr)
    if constexpr (ACC == RES_DOT2) {
      dot2_acc(sr[u], cr[u], a.x, zz.x);
      dot2_acc(sr[u], cr[u], a.y, zz.y);
      dot2_acc(si[u], ci[u], a.x, zz.y);
      dot2_acc(si[u], ci[u], -a.y, zz.x);
    } else if constexpr (ACC == RES_FP64) {
      sr[u] = fma(a.x, zz.x, sr[u]);
      sr[u] = fma(a.y, zz.y, sr[u]);
      si[u] = fma(a.x, zz.y, si[u]);
      si[u] = fma(-a.y, zz.x, si[u]);
    } else {
      const float ar = static_cast<float>(a.x), ai = static_cast<float>(a.y);
      const float zr = static_cast<float>(zz.x), zi = static_cast<float>(zz.y);
      fr[u] = fmaf(ar, zr, fr[u]);
      fr[u] = fmaf(ai, zi, fr[u]);
      fi[u] = fmaf(ar, zi, fi[u]);
      fi[u] = fmaf(-ai, zr, fi[u]);
    }
  };
  if (!C64) {
    // software pipelined: the next row's entries are loaded before the
    // current row's products, and nothing is pending into `a` at loop entry
    double2 a[AHZ_CPW], an[AHZ_CPW];
#pragma unroll
    for (int u = 0; u < AHZ_CPW; ++u)
      a[u] = (cok[u] && lane < rows) ? ld_stream(cp[u] + lane) : make_double2(0.0, 0.0);
    __builtin_amdgcn_s_waitcnt(0);
    for (int i = lane; i < rows; i += 64) {
      const int in = i + 64;
      const bool more = in < rows;
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u)
        an[u] = (cok[u] && more) ? ld_stream(cp[u] + in) : make_double2(0.0, 0.0);
      const double2 zz = zs[i];
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u) acc(u, a[u], zz);
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u) a[u] = an[u];
    }
  } else {
    int i0 = 2 * lane;
    bool done = false;
    {
      // 16-byte aligned A: every entry arrives in a 16-byte load
      // of two adjacent rows, whatever the parity of lda.  Column u's chunk
      // is shifted (sh = 1) when it starts 8 bytes past a 16-byte boundary;
      // its aligned pairs are then rows (1, 2), (3, 4), ... and lane 0 reads
      // row 0 alone.  A column past n reads column 0 of the job and is left
      // out of the sums by a uniform test.  G whole 128-row groups (at
      // either shift), then one group with rows past the chunk zeroed:
      // their loads stay in 16-byte granules that hold a row of the chunk.
      if (r.al16 && rows >= 2) {
        const float2 *cf[AHZ_CPW];
        int sh[AHZ_CPW];
        bool any = false;
#pragma unroll
        for (int u = 0; u < AHZ_CPW; ++u) {
          cf[u] = reinterpret_cast<const float2 *>(cp[u]);
          sh[u] = static_cast<int>((cp[u] - A) & 1);
          any = any || sh[u] != 0;
        }
        const int G = any ? (rows - 1) >> 7 : rows >> 7;
        for (int g = 0; g < G; ++g, i0 += 128) {
          double2 a0[AHZ_CPW], a1[AHZ_CPW];
#pragma unroll
          for (int u = 0; u < AHZ_CPW; ++u) ld_stream_pair(cf[u] + i0 + sh[u], a0[u], a1[u]);
          const double2 z0 = zs[i0], z1 = zs[i0 + 1];
          const double2 z2 = any ? zs[i0 + 2] : z1;
#pragma unroll
          for (int u = 0; u < AHZ_CPW; ++u) {
            if (cok[u]) {
              acc(u, a0[u], sh[u] ? z1 : z0);
              acc(u, a1[u], sh[u] ? z2 : z1);
            }
          }
        }
        {
          double2 a0[AHZ_CPW], a1[AHZ_CPW];
          int f[AHZ_CPW];
#pragma unroll
          for (int u = 0; u < AHZ_CPW; ++u) {
            f[u] = i0 + sh[u];
            ld_stream_pair(cf[u] + (f[u] < rows ? f[u] : sh[u]), a0[u], a1[u]);
          }
#pragma unroll
          for (int u = 0; u < AHZ_CPW; ++u) {
            if (cok[u]) {
              const double2 zero = make_double2(0.0, 0.0);
              const bool v0 = f[u] < rows, v1 = f[u] + 1 < rows;
              acc(u, v0 ? a0[u] : zero, zs[v0 ? f[u] : 0]);
              acc(u, v1 ? a1[u] : zero, zs[v1 ? f[u] + 1 : 0]);
            }
          }
        }
        if (lane == 0) {
#pragma unroll
          for (int u = 0; u < AHZ_CPW; ++u)
            if (cok[u] && sh[u]) acc(u, ld_stream(cp[u]), zs[0]);
        }
        done = true;
      }
    }
    for (int i = i0; !done && i < rows; i += 128) {
      const bool two = i + 1 < rows;
      const double2 z0 = zs[i];
      const double2 z1 = two ? zs[i + 1] : make_double2(0.0, 0.0);
      double2 a0[AHZ_CPW], a1[AHZ_CPW];
#pragma unroll
      for (int u = 0; u < AHZ_CPW; ++u) {
        if (!cok[u]) {
          a0[u] = a1[u] = make_double2(0.0, 0.0);
        } else if (pair && two) {
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
  if constexpr (ACC == RES_FP32) {
#pragma unroll
    for (int u = 0; u < AHZ_CPW; ++u) {
      sr[u] = fr[u];
      si[u] = fi[u];
    }
  }
  // value 2u + p of the reduction: column jb + u, real (p = 0) or imaginary part
  double vs[2 * AHZ_CPW], vc[2 * AHZ_CPW];
#pragma unroll
  for (int u = 0; u < AHZ_CPW; ++u) {
    vs[2 * u] = sr[u];
    vc[2 * u] = cr[u];
    vs[2 * u + 1] = si[u];
    vc[2 * u + 1] = ci[u];
  }
  wave_reduce_dd<2 * AHZ_CPW>(vs, vc);
  constexpr int GROUP = 64 / (2 * AHZ_CPW);
  const int v = lane / GROUP;
  if (lane % GROUP == 0 && jb + (v >> 1) < n) {
    double *o = r.upart + (by * n + jb + (v >> 1)) * 4 + 2 * (v & 1);
    o[0] = vs[0];
    o[1] = vc[0];
  }
}

RID_DEV void u_final_body(const ResJob &r, int64_t bx) {
  if (stopped(r.scal)) return;
  const int64_t j = bx * 256 + threadIdx.x;
  if (j >= r.n) return;
  double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
  // unrolled so that several loads are in flight; the sums keep their order
#pragma unroll 8
  for (int64_t s = 0; s < r.pl.S_u; ++s) {
    const double *o = r.upart + (s * r.n + j) * 4;
    dd_add(sr, cr, o[0], o[1]);
    dd_add(si, ci, o[2], o[3]);
  }
  double hr, lr, hi, li;
  dd_norm(sr, cr, hr, lr);
  dd_norm(si, ci, hi, li);
  r.uh[j] = make_double2(hr, hi);
  r.ul[j] = make_double2(lr, li);
}

// w_j = u_j - sum_t conj(P(t, j)) u_{J[t]}, compensated; x <- w (unscaled).
// Workgroup bx takes columns 64 bx .. 64 bx + 63, one per lane.  u_J is
// staged in LDS 256 rows at a time (a small footprint keeps many
// workgroups resident); wave w takes its quarter of each chunk's rows of P,
// and the four compensated partials are joined in wave order.  The norm
// partial of x is per 64 columns.
RID_DEV void w_body(const ResJob &r, int64_t bx) {
  constexpr int WC = 256;  // rows of u_J per chunk
  __shared__ double2 ujh[WC];
  __shared__ double2 ujl[WC];
  __shared__ double part[4][64][4];
  if (stopped(r.scal)) return;
  const int64_t n = r.n, k = r.k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = bx * 64 + lane;
  double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
  if (j < n && wave == 0) {
    const double2 h = r.uh[j], lo = r.ul[j];
    sr = h.x;
    cr = lo.x;
    si = h.y;
    ci = lo.y;
  }
  const double2 *pc = r.P + (j < n ? j : 0) * r.ldp;
  for (int64_t c0 = 0; c0 < k; c0 += WC) {
    const int64_t kc = min(k - c0, static_cast<int64_t>(WC));
    if (c0 > 0) __syncthreads();  // every wave done with the previous chunk
    if (threadIdx.x < kc) {
      const int64_t jt = r.J[c0 + threadIdx.x];
      const bool ok = jt >= 0 && jt < n;
      ujh[threadIdx.x] = ok ? r.uh[jt] : make_double2(0.0, 0.0);
      ujl[threadIdx.x] = ok ? r.ul[jt] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int64_t kq = (kc + 3) / 4;
    const int64_t t0 = wave * kq, t1 = min(kc, t0 + kq);
    if (j < n) {
#pragma unroll 4
      for (int64_t t = t0; t < t1; ++t) {
        const double2 pe = pc[c0 + t];
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
    }
  }
  part[wave][lane][0] = sr;
  part[wave][lane][1] = cr;
  part[wave][lane][2] = si;
  part[wave][lane][3] = ci;
  __syncthreads();
  if (wave != 0) return;
  double v = 0.0;
  if (j < n) {
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      dd_add(sr, cr, part[w][lane][0], part[w][lane][1]);
      dd_add(si, ci, part[w][lane][2], part[w][lane][3]);
    }
    const double wr = sr + cr, wi = si + ci;
    r.x[j] = make_double2(wr, wi);
    v = wr * wr + wi * wi;
  }
  v = wave_sum(v);
  if (lane == 0) r.wn_part[bx] = v;
}

// ------------------------------------------------------------------ launches
// The steps of the iteration.  Single: the descriptor is the kernel argument
// and the grid is the job's own.  Grouped: block b runs entry tab[b] =
// (job, bx, by) of the step's table.
enum Step : int {
  ST_X0, ST_WNORM, ST_XSCALE, ST_XTINIT, ST_PXP, ST_PXF, ST_AX, ST_ZF, ST_SIGMA, ST_AHZ, ST_UF,
  ST_W, ST_AHZ4, ST_COUNT
};

template <class TA, int STEP, bool WIDE, int ACC, bool GROUPED = false>
RID_DEV void run_step(const ResJob &r, int64_t bx, int64_t by, int t) {
  if constexpr (STEP == ST_X0) x0_body(r, bx);
  if constexpr (STEP == ST_WNORM) wnorm_final_body(r);
  if constexpr (STEP == ST_XSCALE) x_scale_body(r, bx);
  if constexpr (STEP == ST_XTINIT) xt_init_body(r, bx);
  if constexpr (STEP == ST_PXP) px_partial_body(r, bx);
  if constexpr (STEP == ST_PXF) px_final_body(r, bx);
  if constexpr (STEP == ST_AX) {
    // complex64: the paired body with plain sums at any lda, and with
    // compensated sums at an even lda in a batch (one ID keeps the
    // whole-slab fast path below)
    if constexpr (sizeof(TA) == 8 && (ACC != RES_DOT2 || !WIDE)) {
      const bool even = (r.lda & 1) == 0;
      if (r.al16 && r.m >= 2 && (even || (ACC != RES_DOT2 && r.m % r.pl.ax_h != 0))) {
        ax_c64_paired<ACC, GROUPED>(r, bx, by);
        return;
      }
    }
    ax_body<TA, WIDE, ACC>(r, bx, by);
  }
  if constexpr (STEP == ST_ZF) z_final_body(r, bx);
  if constexpr (STEP == ST_SIGMA) sigma_final_body(r, t);
  if constexpr (STEP == ST_AHZ) ahz_body<TA, 8, ACC>(r, bx, by);
  if constexpr (STEP == ST_AHZ4) ahz_body<TA, 4, ACC>(r, bx, by);
  if constexpr (STEP == ST_UF) u_final_body(r, bx);
  if constexpr (STEP == ST_W) w_body(r, bx);
}

template <class TA, int STEP, int ACC>
__global__ __launch_bounds__(256) void step_single(ResJob r, int t) {
  run_step<TA, STEP, true, ACC>(r, blockIdx.x, blockIdx.y, t);
}

template <class TA, int STEP, int ACC>
__global__ __launch_bounds__(256) void step_grouped(const ResJob *__restrict__ jobs,
                                                    const int4 *__restrict__ tab, int t) {
  const int4 e = tab[blockIdx.x];
  // the whole-slab fast path of the ax pass only with plain sums, whose
  // registers leave room for it (with compensated sums it costs a batch
  // more occupancy than its jobs gain)
  run_step<TA, STEP, ACC != RES_DOT2, ACC, true>(jobs[e.x], e.y, e.z, t);
}

// The passes over A take the accumulation `acc` (RES_*); every other step
// has one form.
constexpr bool step_over_A(int step) {
  return step == ST_AX || step == ST_AHZ || step == ST_AHZ4;
}

template <class F>
void by_acc(int step, int acc, F &&f) {
  if (!step_over_A(step) || acc == RES_DOT2)
    f(std::integral_constant<int, RES_DOT2>());
  else if (acc == RES_FP64)
    f(std::integral_constant<int, RES_FP64>());
  else
    f(std::integral_constant<int, RES_FP32>());
}

// blocks of one step for one job (gx by gy)
void step_grid(int step, const ResJob &r, int64_t &gx, int64_t &gy) {
  const ResPlan &p = r.pl;
  gy = 1;
  switch (step) {
    case ST_X0: case ST_XSCALE: case ST_XTINIT: case ST_UF: gx = p.nb_n; break;
    case ST_W: gx = p.nb_w; break;
    case ST_WNORM: case ST_SIGMA: gx = 1; break;
    case ST_PXP: gx = r.k > 0 ? p.nb_pxb : 0; break;
    case ST_PXF: gx = r.k > 0 ? p.nb_k : 0; break;
    case ST_AX: gx = p.nb_ax; gy = p.nb_axy; break;
    case ST_ZF: gx = p.nb_m; break;
    case ST_AHZ: gx = p.ahz_cpw == 8 ? p.nb_ahz : 0; gy = p.S_u; break;
    case ST_AHZ4: gx = p.ahz_cpw == 4 ? p.nb_ahz : 0; gy = p.S_u; break;
    default: gx = 0;
  }
}

template <class TA, int STEP>
void launch_single(hipStream_t st, const ResJob &r, int t, RidProf *prof, int kernel_id) {
  int64_t gx, gy;
  step_grid(STEP, r, gx, gy);
  if (gx * gy == 0) return;
  ProfScope ps(kernel_id >= 0 ? prof : nullptr, st, kernel_id);
  by_acc(STEP, r.acc, [&](auto C) {
    hipLaunchKernelGGL((step_single<TA, STEP, decltype(C)::value>),
                       dim3(static_cast<unsigned>(gx), static_cast<unsigned>(gy)), dim3(256), 0,
                       st, r, t);
  });
}

template <class TA, int STEP>
void launch_grouped(hipStream_t st, const ResJob *jobs, const int4 *tab, int64_t count, int t,
                    int acc, RidProf *prof, int kernel_id) {
  if (count == 0) return;
  ProfScope ps(kernel_id >= 0 ? prof : nullptr, st, kernel_id);
  by_acc(STEP, acc, [&](auto C) {
    hipLaunchKernelGGL((step_grouped<TA, STEP, decltype(C)::value>),
                       dim3(static_cast<unsigned>(count)), dim3(256), 0, st, jobs, tab, t);
  });
}

// The q-step power iteration as a sequence of step launches; L(step, t, id)
// launches one step.
template <class L>
void power_iteration(L &&launch, int q) {
  launch(ST_X0, 0, -1);
  launch(ST_WNORM, 0, -1);
  launch(ST_XSCALE, 0, -1);
  for (int t = 0; t < q; ++t) {
    launch(ST_XTINIT, t, -1);
    launch(ST_PXP, t, -1);
    launch(ST_PXF, t, -1);
    launch(ST_AX, t, RID_KERNEL_AX);
    launch(ST_ZF, t, -1);
    launch(ST_SIGMA, t, -1);
    if (t + 1 < q) {
      launch(ST_AHZ, t, RID_KERNEL_AHZ);   // one of the two has blocks for a job
      launch(ST_AHZ4, t, RID_KERNEL_AHZ);
      launch(ST_UF, t, -1);
      launch(ST_W, t, -1);
      launch(ST_WNORM, t, -1);
      launch(ST_XSCALE, t, -1);
    }
  }
}

// dispatch of a runtime step number to the templated launchers
template <class TA, class F>
void by_step(int step, F &&f) {
  switch (step) {
    case ST_X0: f(std::integral_constant<int, ST_X0>()); break;
    case ST_WNORM: f(std::integral_constant<int, ST_WNORM>()); break;
    case ST_XSCALE: f(std::integral_constant<int, ST_XSCALE>()); break;
    case ST_XTINIT: f(std::integral_constant<int, ST_XTINIT>()); break;
    case ST_PXP: f(std::integral_constant<int, ST_PXP>()); break;
    case ST_PXF: f(std::integral_constant<int, ST_PXF>()); break;
    case ST_AX: f(std::integral_constant<int, ST_AX>()); break;
    case ST_ZF: f(std::integral_constant<int, ST_ZF>()); break;
    case ST_SIGMA: f(std::integral_constant<int, ST_SIGMA>()); break;
    case ST_AHZ: f(std::integral_constant<int, ST_AHZ>()); break;
    case ST_UF: f(std::integral_constant<int, ST_UF>()); break;
    case ST_W: f(std::integral_constant<int, ST_W>()); break;
    case ST_AHZ4: f(std::integral_constant<int, ST_AHZ4>()); break;
    default: break;
  }
}

template <class TA>
void single_iteration(hipStream_t st, const ResJob &r, int q, RidProf *prof) {
  power_iteration(
      [&](int step, int t, int id) {
        by_step<TA>(step, [&](auto S) { launch_single<TA, decltype(S)::value>(st, r, t, prof, id); });
      },
      q);
}

template <class TA>
void grouped_iteration(hipStream_t st, const ResJob *jobs, const int4 *dtab,
                       const GroupedHost &gh, int q, int acc, RidProf *prof) {
  power_iteration(
      [&](int step, int t, int id) {
        by_step<TA>(step, [&](auto S) {
          launch_grouped<TA, decltype(S)::value>(st, jobs, dtab + gh.off[step], gh.cnt[step], t,
                                                 acc, prof, id);
        });
      },
      q);
}

// Rows per ax block for the paired complex64 body of a batch job: the one
// of 512, 256, 128 that pads m least (the larger on a tie), among those it
// can take (an odd lda needs m % h != 0).
int pick_ax_rows(int64_t m, int64_t lda) {
  int best = 0;
  int64_t pad = 0;
  for (int h = AX_ROWS; h >= 128; h >>= 1) {
    if ((lda & 1) && m % h == 0) continue;
    const int64_t p = (m + h - 1) / h * h - m;
    if (best == 0 || p < pad) {
      best = h;
      pad = p;
    }
  }
  return best ? best : AX_ROWS;
}

bool al16_ok(rid_dtype dtype, const void *A) {
  return dtype == RID_C64 && (reinterpret_cast<uintptr_t>(A) % 16 == 0);
}

bool pair_ok(rid_dtype dtype, const void *A, int64_t lda) {
  return dtype == RID_C64 && (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
}

}  // namespace

// ------------------------------------------------------------------ one ID
size_t residual_ws_bytes(int64_t m, int64_t n, int64_t k, int q) {
  (void)q;
  ResJob r{};
  r.m = m;
  r.n = n;
  r.k = k;
  r.pl = plan_res(m, n, k, 2048, 8);
  WsCarve c(nullptr);
  carve_res(c, r);
  return c.off + 256;
}

hipError_t launch_residual(hipStream_t st, rid_dtype dtype, int64_t m, int64_t n, int64_t k,
                           const void *A, int64_t lda, const int64_t *J, const double2 *P,
                           int64_t ldp, int q, uint64_t seed, double *sigma, double *hist,
                           void *ws, RidProf *prof, int acc) {
  if (k > RES_KMAX) return hipErrorInvalidValue;
  ResJob r{};
  r.acc = acc;
  r.m = m;
  r.n = n;
  r.k = k;
  r.lda = lda;
  r.ldp = ldp;
  r.A = A;
  r.J = J;
  r.P = P;
  r.seed = seed;
  r.sigma = sigma;
  r.hist = hist;
  r.pair = pair_ok(dtype, A, lda) ? 1 : 0;
  r.al16 = al16_ok(dtype, A) ? 1 : 0;
  r.pl = plan_res(m, n, k, 2048, dtype == RID_C64 ? 4 : 8);
  WsCarve c(ws);
  carve_res(c, r);
  if (dtype == RID_C64)
    single_iteration<float2>(st, r, q, prof);
  else
    single_iteration<double2>(st, r, q, prof);
  return hipGetLastError();
}

// ------------------------------------------------------------------ a batch of IDs
void residual_batch_setup(const RidBatchJob *bj, int count, rid_dtype dtype, int64_t block_bytes,
                          int ahz_cpw, int acc, void *ws, GroupedHost *out) {
  WsCarve c(ws);
  if (block_bytes < 1) block_bytes = 1;
  std::vector<ResJob> jobs(count);
  for (int i = 0; i < count; ++i) {
    ResJob &r = jobs[i];
    r = ResJob{};
    r.acc = acc;
    r.m = bj[i].m;
    r.n = bj[i].n;
    r.k = bj[i].k;
    r.lda = bj[i].lda;
    r.ldp = bj[i].ldp;
    r.A = bj[i].A;
    r.J = bj[i].J;
    r.P = bj[i].P;
    r.seed = bj[i].seed;
    r.sigma = bj[i].sigma;
    r.hist = nullptr;
    r.pair = pair_ok(dtype, bj[i].A, bj[i].lda) ? 1 : 0;
    r.al16 = al16_ok(dtype, bj[i].A) ? 1 : 0;
    // a job's own passes need few workgroups (the batch fills the device):
    // about one ax workgroup per block_bytes of A
    const int64_t abytes = r.m * r.n * (dtype == RID_C64 ? 8 : 16);
    r.pl = plan_res(r.m, r.n, r.k,
                    std::min<int64_t>(2048, std::max<int64_t>(1, abytes / block_bytes)), ahz_cpw);
    if (dtype == RID_C64 && r.al16 && r.m >= 2 && (acc != RES_DOT2 || (r.lda & 1) == 0))
      set_ax_rows(r.pl, r.m, pick_ax_rows(r.m, r.lda));
    carve_res(c, r);
  }
  out->ws_bytes = c.off + 256;
  out->jobs.resize(sizeof(ResJob) * count);
  if (count) memcpy(out->jobs.data(), jobs.data(), sizeof(ResJob) * count);
  out->tab.clear();
  for (int s = 0; s < ST_COUNT; ++s) {
    out->off[s] = static_cast<int64_t>(out->tab.size());
    for (int i = 0; i < count; ++i) {
      int64_t gx, gy;
      step_grid(s, jobs[i], gx, gy);
      for (int64_t y = 0; y < gy; ++y)
        for (int64_t x = 0; x < gx; ++x)
          out->tab.push_back(make_int4(i, static_cast<int>(x), static_cast<int>(y), 0));
    }
    out->cnt[s] = static_cast<int64_t>(out->tab.size()) - out->off[s];
  }
}

hipError_t launch_residual_batch(hipStream_t st, rid_dtype dtype, const void *djobs,
                                 const int4 *dtab, const GroupedHost &gh, int q, int acc,
                                 RidProf *prof) {
  const ResJob *jobs = static_cast<const ResJob *>(djobs);
  if (dtype == RID_C64)
    grouped_iteration<float2>(st, jobs, dtab, gh, q, acc, prof);
  else
    grouped_iteration<double2>(st, jobs, dtab, gh, q, acc, prof);
  return hipGetLastError();
}
