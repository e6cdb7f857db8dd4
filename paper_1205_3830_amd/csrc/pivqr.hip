// pivqr.hip -- column-pivoted Householder QR of the l x n sketch Y, the
// approximate QR with column permutation of Sec. 2.  Only the first k steps
// are taken; the pivots are the skeleton J.
//
// One kernel per step.  Workgroup b (4 waves) owns columns [64b, 64b + 64),
// each wave 16 of them, one column at a time with the rows spread over the
// 64 lanes (RR rows per lane, l <= 64 RR <= 2048).  Kernel t
//   1. merges the per-workgroup candidates of step t-1 into the pivot j* of
//      step t-1 (max trailing norm, lowest index on exact ties) -- every
//      workgroup does the same merge in the same order, so all agree;
//   2. rebuilds the Householder reflector of step t-1 from the candidate
//      copy of column j* (LAPACK zlarfg convention, real diagonal beta) and
//      applies its adjoint to the rows t-1.. of its own unpicked columns;
//      the owner of j* writes beta and zeros into that column;
//   3. recomputes the exact trailing norm (rows t..l-1) of each unpicked
//      column and publishes its best column (norm, index, a copy of the
//      trailing rows) and second-best norm for step t.
// Columns stay in place: after the last kernel, Y(0:k, :) is R in original
// column order.  No floating-point atomics; every reduction has a fixed order.
#include <algorithm>
#include <cstdlib>
#include <climits>
#include <type_traits>

#include "rid_internal.hpp"

namespace {

constexpr int PQ_COLS = 64;

// The per-workgroup candidates are double-buffered by step parity: launch t
// reads the candidates of step t-1 (buffer (t-1) & 1) to rebuild the
// reflector and writes those of step t (buffer t & 1).  With one buffer, a
// workgroup that finishes early would overwrite the pivot column's copy
// while workgroups that start later (when there are more than fit on the
// device at once) still have to read it.
struct PivWs {
  double *cnorm;   // [2][nb] best trailing norm of the block (-1: none)
  double *cnorm2;  // [2][nb] its second-best norm (-1: none)
  int64_t *cidx;   // [2][nb] column index of the best
  double2 *ccol;   // [2][nb][l] copy of the best column (rows t..l-1 valid)
  int *pstep;      // [n] step at which the column was picked, -1 if not
  double *nu0;     // best norm of step 0
};

PivWs carve_piv(void *ws, int64_t l, int64_t n) {
  WsCarve c(ws);
  const int64_t nb = (n + PQ_COLS - 1) / PQ_COLS;
  PivWs w;
  w.cnorm = c.take<double>(2 * nb);
  w.cnorm2 = c.take<double>(2 * nb);
  w.cidx = c.take<int64_t>(2 * nb);
  w.ccol = c.take<double2>(2 * size_t(nb) * size_t(l));
  w.pstep = c.take<int>(n);
  w.nu0 = c.take<double>(1);
  return w;
}

size_t piv_bytes(int64_t l, int64_t n) {
  WsCarve c(nullptr);
  const int64_t nb = (n + PQ_COLS - 1) / PQ_COLS;
  c.take<double>(2 * nb);
  c.take<double>(2 * nb);
  c.take<int64_t>(2 * nb);
  c.take<double2>(2 * size_t(nb) * size_t(l));
  c.take<int>(n);
  c.take<double>(1);
  return c.off + 256;
}

// (best value, its column, second-best value); larger value wins, lower
// column index wins an exact tie.
struct Cand {
  double v1;
  int64_t i1;
  double v2;
  int src;  // wave that holds the best (block-level merge only)
};

RID_DEV Cand cand_empty() { return Cand{-1.0, LLONG_MAX, -1.0, -1}; }

RID_DEV Cand cand_merge(Cand a, Cand b) {
  const bool bwins = (b.v1 > a.v1) || (b.v1 == a.v1 && b.i1 < a.i1);
  Cand w = bwins ? b : a;
  const Cand o = bwins ? a : b;
  w.v2 = fmax(w.v2, o.v1);
  return w;
}

// The candidate of lane (lane op CTRL) for a DPP pattern CTRL (src, the
// same in every lane of a wave wherever this is used, stays).
template <int CTRL>
RID_DEV Cand cand_dpp(const Cand &c) {
  return Cand{dpp_f64<CTRL>(c.v1), dpp_i64<CTRL>(c.i1), dpp_f64<CTRL>(c.v2), c.src};
}

template <int W>
RID_DEV Cand cand_swap_merge(const Cand &c) {
  Cand a, b;
  swap_pair<W>(c.v1, a.v1, b.v1);
  swap_pair<W>(c.i1, a.i1, b.i1);
  swap_pair<W>(c.v2, a.v2, b.v2);
  a.src = b.src = c.src;
  return cand_merge(a, b);
}

// The merge of the 64 lanes' candidates, in every lane.  cand_merge is
// symmetric (the winner and the largest other value do not depend on the
// order), so the butterfly of wave_sum applies: both copies of the lane-swap
// levels are merged, and the row rotations and quad patterns read a lane
// that holds the partner's candidate.  No LDS traffic and no barrier.
RID_DEV Cand cand_wave_merge(Cand c) {
  c = cand_swap_merge<32>(c);
  c = cand_swap_merge<16>(c);
  c = cand_merge(c, cand_dpp<0x128>(c));  // row_ror:8
  c = cand_merge(c, cand_dpp<0x124>(c));  // row_ror:4
  c = cand_merge(c, cand_dpp<0x4E>(c));   // quad_perm [2,3,0,1]
  c = cand_merge(c, cand_dpp<0xB1>(c));   // quad_perm [1,0,3,2]
  return c;
}

// The merge of a 256-thread workgroup's candidates, the same in every
// thread: each wave's merge, then the four in wave order.  red holds at least
// four candidates in LDS; the caller writes none of red[0..3] again before a
// barrier that every thread reaches after this call.
RID_DEV Cand cand_block_merge(Cand cd, Cand *red) {
  cd = cand_wave_merge(cd);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cd;
  __syncthreads();
  Cand best = cand_empty();
#pragma unroll
  for (int wv = 0; wv < 4; ++wv) best = cand_merge(best, red[wv]);
  return best;
}

__global__ void pivqr_init_kernel(int64_t n, int *pstep, int *status) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j < n) pstep[j] = -1;
  if (j == 0) *status = RID_OK;
}

// Step t of the QR for workgroup bx of nb (the column owner of [64 bx, 64 bx + 64)).
// A wave handles CB of its 16 columns at a time.
// Buffer loads and stores as buf_ld / buf_st, with the non-temporal hint
// (cache policy bit 1): for a Y far beyond the caches, which every step
// streams once.
RID_DEV double2 buf_ld_nt(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 2));
}
RID_DEV void buf_st_nt(__amdgpu_buffer_rsrc_t r, int off, double2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 2);
}


// Independent FMA chains per lane sum: row h of a lane goes to chain h % NC,
// and the chains are added pairwise at the end.  With one wave per SIMD (the
// large-l steps) nothing else hides a chain's latency, so four overlapping
// chains of RR/4 terms replace one of RR.
template <int RR>
constexpr int lane_chains() {
  return RR < 4 ? RR : 4;
}
template <int NC>
RID_DEV double add_chains(const double (&c)[NC]) {
  if constexpr (NC == 4) return (c[0] + c[1]) + (c[2] + c[3]);
  if constexpr (NC == 3) return (c[0] + c[1]) + c[2];
  if constexpr (NC == 2) return c[0] + c[1];
  return c[0];
}

// Sum of |y_h|^2 over the lane's RR rows, row 0 only when `first`.
template <int RR>
RID_DEV double rows_norm2(const double2 (&y)[RR], bool first) {
  constexpr int NC = lane_chains<RR>();
  double c[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) c[i] = 0.0;
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const double2 q = (h > 0 || first) ? y[h] : make_double2(0.0, 0.0);
    c[h % NC] = fma(q.x, q.x, c[h % NC]);
    c[h % NC] = fma(q.y, q.y, c[h % NC]);
  }
  return add_chains<NC>(c);
}

// y_b -= conj(tau) (v^H y_b) v for CB columns over the lane's RR rows, with
// one LDS read of v per row for all of them; bit b of zmask gives column b a
// zero coefficient (it is left as it is).  Sums (in lane_chains chains) and
// updates are plain FMA chains, the same for every column.
template <int RR, int CB>
RID_DEV void apply_reflector(double2 (&y)[CB][RR], const double2 *vl, double2 tau, int lane,
                         unsigned zmask) {
  constexpr int NC = lane_chains<RR>();
  double pr[CB][NC], pi[CB][NC];
#pragma unroll
  for (int b = 0; b < CB; ++b)
#pragma unroll
    for (int i = 0; i < NC; ++i) pr[b][i] = pi[b][i] = 0.0;
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const double2 v = vl[lane + 64 * h];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      double &r = pr[b][h % NC], &i = pi[b][h % NC];
      r = fma(v.x, y[b][h].x, r);
      r = fma(v.y, y[b][h].y, r);
      i = fma(v.x, y[b][h].y, i);
      i = fma(-v.y, y[b][h].x, i);
    }
  }
  double dr[CB], di[CB], cr[CB], ci[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    dr[b] = wave_sum(add_chains<NC>(pr[b]));
    di[b] = wave_sum(add_chains<NC>(pi[b]));
    const bool z = (zmask >> b) & 1u;
    cr[b] = z ? 0.0 : tau.x * dr[b] + tau.y * di[b];
    ci[b] = z ? 0.0 : tau.x * di[b] - tau.y * dr[b];
  }
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const double2 v = vl[lane + 64 * h];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      y[b][h].x = fma(-v.x, cr[b], y[b][h].x);
      y[b][h].x = fma(v.y, ci[b], y[b][h].x);
      y[b][h].y = fma(-v.x, ci[b], y[b][h].y);
      y[b][h].y = fma(-v.y, cr[b], y[b][h].y);
    }
  }
}

// The Householder reflector (zlarfg convention: real beta, v(0) = 1) that
// maps rows r0 .. l-1 of column x (x indexed by absolute row) to beta e_0,
// built by one wave: v into v_s (rows relative to r0, zero past l), tau and
// beta into tau_s and beta_s.
template <int RR>
RID_DEV void make_reflector(const double2 *x, int64_t r0, int64_t l, int lane, double2 *v_s,
                            double2 &tau_s, double &beta_s) {
  double2 xv[RR];
  double ss = 0.0;
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const int64_t row = r0 + lane + 64 * h;
    xv[h] = (row < l) ? x[row] : make_double2(0.0, 0.0);
    if (lane + 64 * h >= 1) ss += xv[h].x * xv[h].x + xv[h].y * xv[h].y;
  }
  const double xnorm2 = wave_sum(ss);
  const double ar = lane_bcast(xv[0].x, 0);
  const double ai = lane_bcast(xv[0].y, 0);
  double2 tau;
  double beta;
  double2 scale;
  if (xnorm2 == 0.0 && ai == 0.0) {
    tau = make_double2(0.0, 0.0);
    beta = ar;
    scale = make_double2(0.0, 0.0);
  } else {
    const double mag = sqrt(ar * ar + ai * ai + xnorm2);
    beta = (ar >= 0.0) ? -mag : mag;
    tau = make_double2((beta - ar) / beta, -ai / beta);
    // scale = 1 / (alpha - beta)
    const double dr = ar - beta, di = ai;
    const double den = dr * dr + di * di;
    scale = make_double2(dr / den, -di / den);
  }
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const int idx = lane + 64 * h;
    double2 v;
    if (idx == 0) {
      v = make_double2(1.0, 0.0);
    } else {
      v = make_double2(xv[h].x * scale.x - xv[h].y * scale.y,
                       xv[h].x * scale.y + xv[h].y * scale.x);
    }
    v_s[idx] = (r0 + idx < l) ? v : make_double2(0.0, 0.0);
  }
  if (lane == 0) {
    tau_s = tau;
    beta_s = beta;
  }
}

template <int RR, int CB>
RID_DEV void pivqr_step_body(int t, int64_t l, int64_t n, int64_t k, double2 *Y, int64_t ldy,
                             int64_t *perm, double *gaps, double rank_tol, const PivWs &w,
                             int *status, int64_t bx, int64_t nb) {
  __shared__ double2 v_s[64 * RR];
  __shared__ Cand red[4];
  __shared__ double2 tau_s;
  __shared__ double beta_s;
  __shared__ int status_s;

  // workgroup 0 of this same launch may be writing the status word: one
  // read, shared, so that the whole workgroup leaves or stays together
  if (threadIdx.x == 0) status_s = *status;
  __syncthreads();
  if (status_s != RID_OK) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // uniform in the wave; read as such, so that buffer resources built from
  // it stay in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t cbeg = bx * PQ_COLS;
  int64_t jstar = -1;
  const int64_t r0 = (t > 0) ? t - 1 : 0;  // first row touched by this kernel

  const int64_t rd = ((t - 1) & 1) * nb;  // candidates of step t-1
  const int64_t wr = (t & 1) * nb;        // candidates of step t
  if (t > 0) {
    // ---- 1. pivot of step t-1
    Cand cd = cand_empty();
    for (int64_t b = tid; b < nb; b += 256) {
      Cand x{w.cnorm[rd + b], w.cidx[rd + b], w.cnorm2[rd + b], 0};
      if (x.v1 < 0.0) x = cand_empty();
      cd = cand_merge(cd, x);
    }
    // the same in every lane: read as uniform, so that what depends on it
    // (the exit on failure, the pivot index) stays uniform for the compiler
    Cand best = cand_block_merge(cd, red);
    best.v1 = uniform_f64(best.v1);
    best.i1 = uniform_i64(best.i1);
    const double nu1 = best.v1;
    const double nu0 = (t == 1) ? nu1 : *w.nu0;
    const bool fail = !(nu1 > 0.0) || nu1 <= rank_tol * nu0;
    if (bx == 0 && tid == 0) {
      perm[t - 1] = best.i1;
      if (gaps) gaps[t - 1] = (best.v2 < 0.0) ? 1.0 : (nu1 - best.v2) / nu1;
      if (t == 1) *w.nu0 = nu1;
      if (fail) *status = RID_ERR_RANK;
    }
    if (fail) return;
    jstar = best.i1;
    const int64_t bstar = jstar / PQ_COLS;

    // ---- 2. reflector of step t-1 from the candidate copy (wave 0)
    if (wave == 0) make_reflector<RR>(w.ccol + (rd + bstar) * l, r0, l, lane, v_s, tau_s, beta_s);
    __syncthreads();
  }

  // ---- 2b/3. apply the reflector, then the trailing norms of step t.  A
  // column slice is rows r0 .. l-1 through a range-checked buffer resource:
  // rows past l load as zeros (as v holds there) and are never stored.
  const double2 tau = (t > 0) ? tau_s : make_double2(0.0, 0.0);
  const double beta = (t > 0) ? beta_s : 0.0;
  const int64_t jw = cbeg + wave * 16;
  const int64_t jp = uniform_i64(jstar);  // scalar, as the buffer resources need
  // picked-step marks of the wave's 16 columns, read at once: bit c is set
  // for an unpicked column (the pivot of step t-1 included)
  const bool inr = lane < 16 && jw + lane < n;
  const uint64_t open = __ballot(inr && w.pstep[inr ? jw + lane : 0] < 0);
  const int nbytes = static_cast<int>((l - r0) * 16);
  const int lo = lane * 16;
  Cand wc = cand_empty();
  // CB columns at a time: their loads, reductions and stores are independent
  // chains that overlap; each column's own arithmetic and reduction order is
  // the same as one column at a time, so the results are too.  The merge of
  // candidates is independent of order (max value, lowest index on ties).
  for (int c0 = 0; c0 < 16; c0 += CB) {
    double2 y[CB][RR];
    __amdgpu_buffer_rsrc_t rs[CB];
    bool live[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int64_t j = jw + c0 + b;
      const bool open_j = (open >> (c0 + b)) & 1;
      if (open_j && j == jp) {
        // the pivot of step t-1: beta at row r0, zeros below
        const __amdgpu_buffer_rsrc_t rp = buf_rsrc(Y + j * ldy + r0, nbytes);
#pragma unroll
        for (int h = 0; h < RR; ++h)
          buf_st(rp, lo + 1024 * h,
                 (h == 0 && lane == 0) ? make_double2(beta, 0.0) : make_double2(0.0, 0.0));
        if (lane == 0) w.pstep[j] = t - 1;
      }
      live[b] = open_j && j != jp;
      rs[b] = buf_rsrc(live[b] ? Y + j * ldy + r0 : Y, live[b] ? nbytes : 0);
#pragma unroll
      for (int h = 0; h < RR; ++h) y[b][h] = buf_ld(rs[b], lo + 1024 * h);
    }
    if (t > 0) {
      apply_reflector<RR, CB>(y, v_s, tau, lane, 0u);
#pragma unroll
      for (int b = 0; b < CB; ++b)
#pragma unroll
        for (int h = 0; h < RR; ++h) buf_st(rs[b], lo + 1024 * h, y[b][h]);
    }
    if (t < k) {
      // rows t .. l-1: all but row r0 = t-1 (lane 0 of slot 0) when t > 0
      const bool below = lane >= t - r0;
      double ss[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) ss[b] = rows_norm2<RR>(y[b], below);
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const double nrm = sqrt(wave_sum(ss[b]));
        if (live[b]) wc = cand_merge(wc, Cand{nrm, jw + c0 + b, -1.0, wave});
      }
    }
  }
  if (t >= k) return;

  // ---- block-level candidate, merged in wave order
  if (lane == 0) red[wave] = wc;
  __syncthreads();
  Cand bc = cand_empty();
  for (int wv = 0; wv < 4; ++wv) bc = cand_merge(bc, red[wv]);
  if (tid == 0) {
    w.cnorm[wr + bx] = bc.v1;
    w.cnorm2[wr + bx] = bc.v2;
    w.cidx[wr + bx] = bc.i1;
  }
  // publish a copy of the block's best column, re-read from Y: its owning
  // wave stored it (updated) before the barrier above
  if (bc.src >= 0) {
    const double2 *src = Y + bc.i1 * ldy;
    double2 *dst = w.ccol + (wr + bx) * l;
    for (int64_t row = t + tid; row < l; row += 256) dst[row] = src[row];
  }
}

// ---------------------------------------------------------------- panel form
// For a Y much larger than the last-level cache (8.4 GB at 2000 x 2^18) each
// step of the plain kernel re-reads and rewrites the trailing rows.  The panel
// form keeps up to QP_NB reflectors pending.  Step t applies the pending
// reflectors a .. t-1 to each unpicked column in registers, in order and each
// as in the plain kernel, takes the exact trailing norms from the result, and
// writes the updated rows back only when the panel is full (t - a = QP_NB) or
// at the last step; so the pivots are chosen on exact norms as before.  The
// pivot column is written at its own step: the pending reflectors a .. t-2
// applied to its rows a .. t-2 (its entries of R), beta at row t-1, zeros
// below.  Reflector s is kept, full length and zero above row s, in global
// slot s % QP_NB (written by workgroup 0 when it is built); each step loads
// the pending ones into LDS, rows relative to a.  When a step writes nothing,
// the owning wave of a block's best column recomputes it (re-read, pending
// reflectors applied) for the candidate copy.
constexpr int QP_NB = 4;

struct PanelWs {
  double2 *V;    // [QP_NB][l] reflector slots
  double2 *tau;  // [QP_NB]
};

// A workgroup takes the column blocks slot, slot + G, ... (G = gridDim.x,
// sized to the workgroups the device holds at once), so the per-step work
// of a workgroup -- merging the previous step's candidates, building the
// reflector, staging the pending reflectors -- is done once for all of its
// blocks, and it publishes one candidate (its best column) in slot `slot`.
// nbk: column blocks; gprev: candidate slots the previous step wrote.
template <int RR, int CB>
__global__ __launch_bounds__(256) void pivqr_panel_kernel(int t, int a, int wr, int64_t l,
                                                          int64_t n, int64_t k, double2 *Y,
                                                          int64_t ldy, int64_t *perm,
                                                          double *gaps, double rank_tol,
                                                          PivWs w, PanelWs pw, int *status,
                                                          int64_t nbk, int64_t gprev) {
  __shared__ double2 vl[QP_NB][64 * RR];
  __shared__ double2 taus[QP_NB];
  __shared__ Cand red[4];
  __shared__ double beta_s;
  __shared__ int status_s;
  if (threadIdx.x == 0) status_s = *status;
  __syncthreads();
  if (status_s != RID_OK) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // uniform in the wave; read as such, so that buffer resources built from
  // it stay in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t slot = blockIdx.x;
  const int64_t G = gridDim.x;
  const int64_t rd = ((t - 1) & 1) * nbk;  // candidates of step t-1
  const int64_t wrb = (t & 1) * nbk;       // candidates of step t
  int64_t jstar = -1;
  double beta = 0.0;
  // the pending reflectors a .. t-2, rows relative to a
  for (int s = a; s < t - 1; ++s) {
    const int sl = s % QP_NB;
    for (int idx = tid; idx < 64 * RR; idx += 256) {
      const int64_t row = a + idx;
      vl[sl][idx] = (row < l) ? pw.V[sl * l + row] : make_double2(0.0, 0.0);
    }
    if (tid == 0) taus[sl] = pw.tau[sl];
  }
  if (t > 0) {
    // ---- pivot of step t-1 (as in the plain kernel)
    Cand cd = cand_empty();
    for (int64_t b = tid; b < gprev; b += 256) {
      Cand x{w.cnorm[rd + b], w.cidx[rd + b], w.cnorm2[rd + b], 0};
      if (x.v1 < 0.0) x = cand_empty();
      cd = cand_merge(cd, x);
    }
    // the same in every lane: read as uniform, so that what depends on it
    // (the exit on failure, the pivot index) stays uniform for the compiler
    Cand best = cand_block_merge(cd, red);
    best.v1 = uniform_f64(best.v1);
    best.i1 = uniform_i64(best.i1);
    const double nu1 = best.v1;
    const double nu0 = (t == 1) ? nu1 : *w.nu0;
    const bool fail = !(nu1 > 0.0) || nu1 <= rank_tol * nu0;
    if (slot == 0 && tid == 0) {
      perm[t - 1] = best.i1;
      if (gaps) gaps[t - 1] = (best.v2 < 0.0) ? 1.0 : (nu1 - best.v2) / nu1;
      if (t == 1) *w.nu0 = nu1;
      if (fail) *status = RID_ERR_RANK;
    }
    if (fail) return;
    jstar = best.i1;
    // ---- reflector of step t-1 from the candidate copy (wave 0), into slot
    // (t-1) % QP_NB: rows a .. t-2 zero, 1 at row t-1, the scaled copy below
    const int sl = (t - 1) % QP_NB;
    if (wave == 0) {
      const int64_t r0 = t - 1;
      // the copy sits in the slot of the workgroup that took j*'s block
      const double2 *x = w.ccol + (rd + (jstar / PQ_COLS) % gprev) * l;
      double2 xv[RR];
      double ss = 0.0;
#pragma unroll
      for (int h = 0; h < RR; ++h) {
        const int64_t row = r0 + lane + 64 * h;
        xv[h] = (row < l) ? x[row] : make_double2(0.0, 0.0);
        if (lane + 64 * h >= 1) ss += xv[h].x * xv[h].x + xv[h].y * xv[h].y;
      }
      const double xnorm2 = wave_sum(ss);
      const double ar = lane_bcast(xv[0].x, 0);
      const double ai = lane_bcast(xv[0].y, 0);
      double2 tau;
      double2 scale;
      if (xnorm2 == 0.0 && ai == 0.0) {
        tau = make_double2(0.0, 0.0);
        beta = ar;
        scale = make_double2(0.0, 0.0);
      } else {
        const double mag = sqrt(ar * ar + ai * ai + xnorm2);
        beta = (ar >= 0.0) ? -mag : mag;
        tau = make_double2((beta - ar) / beta, -ai / beta);
        const double dr = ar - beta, di = ai;
        const double den = dr * dr + di * di;
        scale = make_double2(dr / den, -di / den);
      }
      for (int64_t idx = lane; idx < 64 * RR; idx += 64) vl[sl][idx] = make_double2(0.0, 0.0);
#pragma unroll
      for (int h = 0; h < RR; ++h) {
        const int idx = lane + 64 * h;
        const int64_t row = r0 + idx;
        if (row < l) {
          const double2 v = (idx == 0) ? make_double2(1.0, 0.0)
                                       : make_double2(xv[h].x * scale.x - xv[h].y * scale.y,
                                                      xv[h].x * scale.y + xv[h].y * scale.x);
          vl[sl][row - a] = v;
          if (slot == 0) pw.V[sl * l + row] = v;
        }
      }
      if (slot == 0)
        for (int64_t row = lane; row < r0; row += 64) pw.V[sl * l + row] = make_double2(0.0, 0.0);
      if (lane == 0) {
        taus[sl] = tau;
        beta_s = beta;
        if (slot == 0) pw.tau[sl] = tau;
      }
    }
    __syncthreads();
    beta = beta_s;
  } else {
    __syncthreads();
  }

  // ---- the columns, CB at a time: pending reflectors in order, then the
  // exact trailing norm.  A reflector is read from LDS once for the CB
  // columns, and their reduction chains overlap; each column's operations
  // are those of one column alone (the pivot column of step t-1 takes a zero
  // coefficient for reflector t-1).  A column slice is rows a .. l-1 through
  // a range-checked buffer resource: rows past l load as zeros (and stay
  // zero, as do the reflectors there) and are never stored.
  const int nbytes = static_cast<int>((l - a) * 16);
  const int lo = lane * 16;
  Cand wc = cand_empty();
  for (int64_t bx = slot; bx < nbk; bx += G) {
    const int64_t jw = bx * PQ_COLS + wave * 16;
    // picked-step marks of the wave's 16 columns, read at once: bit c is set
    // for an unpicked column (the pivot of step t-1 included)
    const bool inr = lane < 16 && jw + lane < n;
    const uint64_t open = __ballot(inr && w.pstep[inr ? jw + lane : 0] < 0);
    for (int c0 = 0; c0 < 16; c0 += CB) {
      double2 y[CB][RR];
      __amdgpu_buffer_rsrc_t rs[CB];
      bool live[CB];
      unsigned zmask = 0;
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int64_t j = jw + c0 + b;
        live[b] = (open >> (c0 + b)) & 1;
        if (j == jstar) zmask |= 1u << b;
        rs[b] = buf_rsrc(live[b] ? Y + j * ldy + a : Y, live[b] ? nbytes : 0);
#pragma unroll
        for (int h = 0; h < RR; ++h) y[b][h] = buf_ld_nt(rs[b], lo + 1024 * h);
      }
      for (int s = a; s < t; ++s)
        apply_reflector<RR, CB>(y, vl[s % QP_NB], taus[s % QP_NB], lane,
                                (s == t - 1) ? zmask : 0u);
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        if (!live[b]) continue;
        if ((zmask >> b) & 1u) {
          // rows a .. t-2: its entries of R; beta at row t-1; zeros below
#pragma unroll
          for (int h = 0; h < RR; ++h) {
            const int64_t row = a + lane + 64 * h;
            const double2 v = (row < t - 1) ? y[b][h]
                                            : ((row == t - 1) ? make_double2(beta, 0.0)
                                                              : make_double2(0.0, 0.0));
            buf_st_nt(rs[b], lo + 1024 * h, v);
          }
          if (lane == 0) w.pstep[jw + c0 + b] = t - 1;
        } else if (wr) {
#pragma unroll
          for (int h = 0; h < RR; ++h) buf_st_nt(rs[b], lo + 1024 * h, y[b][h]);
        }
      }
      if (t < k) {
        // rows t .. l-1: all but rows a .. t-1, which sit in slot 0
        const bool below = lane >= t - a;
        double ss[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) ss[b] = rows_norm2<RR>(y[b], below);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
          const double nrm = sqrt(wave_sum(ss[b]));
          if (live[b] && !((zmask >> b) & 1u))
            wc = cand_merge(wc, Cand{nrm, jw + c0 + b, -1.0, wave});
        }
      }
    }
  }
  if (t >= k) return;

  // ---- workgroup-level candidate, merged in wave order
  if (lane == 0) red[wave] = wc;
  __syncthreads();
  Cand bc = cand_empty();
  for (int wv = 0; wv < 4; ++wv) bc = cand_merge(bc, red[wv]);
  if (tid == 0) {
    w.cnorm[wrb + slot] = bc.v1;
    w.cnorm2[wrb + slot] = bc.v2;
    w.cidx[wrb + slot] = bc.i1;
  }
  if (bc.src < 0) return;
  double2 *dst = w.ccol + (wrb + slot) * l;
  if (wr || t == a) {
    // Y holds the column as of this step (written above, or nothing pending)
    const double2 *src = Y + bc.i1 * ldy;
    for (int64_t row = t + tid; row < l; row += 256) dst[row] = src[row];
  } else if (wave == bc.src) {
    // the same loads and arithmetic as in the column loop above
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(Y + uniform_i64(bc.i1) * ldy + a, nbytes);
    double2 y[1][RR];
#pragma unroll
    for (int h = 0; h < RR; ++h) y[0][h] = buf_ld(rs, lo + 1024 * h);
    for (int s = a; s < t; ++s) apply_reflector<RR, 1>(y, vl[s % QP_NB], taus[s % QP_NB], lane, 0u);
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t row = a + lane + 64 * h;
      if (row >= t && row < l) dst[row] = y[0][h];
    }
  }
}

template <int RR, int CB>
__global__ __launch_bounds__(256) void pivqr_step_kernel(int t, int64_t l, int64_t n,
                                                         int64_t k, double2 *Y, int64_t ldy,
                                                         int64_t *perm, double *gaps,
                                                         double rank_tol, PivWs w,
                                                         int *status) {
  pivqr_step_body<RR, CB>(t, l, n, k, Y, ldy, perm, gaps, rank_tol, w, status, blockIdx.x,
                          gridDim.x);
}

// A batch: block b is column block tab[b].y of job tab[b].x (tab[b].z blocks
// in that job).  Jobs with k < t have finished and leave at once.
template <int RR, int CB>
__global__ __launch_bounds__(256) void pivqr_step_grouped(int t, const PivJob *__restrict__ jobs,
                                                          const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const PivJob &jb = jobs[e.x];
  if (t > jb.k) return;
  const PivWs w{jb.cnorm, jb.cnorm2, jb.cidx, jb.ccol, jb.mark, jb.nu0};
  // a batch fills the device with workgroups: one column at a time keeps
  // the registers, and so the occupancy, of the plain loop
  pivqr_step_body<RR, CB>(t, jb.l, jb.n, jb.k, jb.Y, jb.ldy, jb.J, nullptr, jb.rank_tol, w,
                         jb.status, e.y, e.z);
}

// A batch: the picked-step marks of each job's own columns start at -1; the
// first block of a job also clears its status word.
__global__ __launch_bounds__(256) void pivqr_init_grouped(const PivJob *__restrict__ jobs,
                                                          const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const PivJob &jb = jobs[e.x];
  if (threadIdx.x < PQ_COLS) {
    const int64_t j = int64_t(e.y) * PQ_COLS + threadIdx.x;
    if (j < jb.n) jb.mark[j] = -1;
  }
  if (e.y == 0 && threadIdx.x == 0) *jb.status = RID_OK;
}

// ---------------------------------------------------------------- a batch, one workgroup per job
// Every step of one job's QR runs in one workgroup of PJ_WAVES waves, which
// keeps the job's pivot candidates and reflector in LDS from step to step:
// the QR of the whole batch is one launch (a workgroup per job, largest
// jobs first), in which a job moves to its next step as soon as its own
// columns are done, whatever the other jobs do.  Wave w owns the columns
// CB w + 16 CB i + b (b < CB) for all steps.  The per-column arithmetic --
// the reflector, its update and the trailing norms -- is that of
// pivqr_step_body, and the candidate merge takes the same maximum (lowest
// index on exact ties), so J and R equal the per-step launches' bit for bit.
constexpr int PJ_WAVES = 16;

template <int RR, int CB>
RID_DEV void pivqr_job_body(const PivJob &jb, double2 *v_s, Cand *red, double2 &tau_s,
                            double &beta_s) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t l = jb.l, n = jb.n, k = jb.k, ldy = jb.ldy;
  double2 *Y = jb.Y;
  int *mark = jb.mark;
  for (int64_t j = tid; j < n; j += blockDim.x) mark[j] = -1;
  if (tid == 0) *jb.status = RID_OK;
  __syncthreads();
  double nu0 = 0.0;
  int64_t jstar = -1;
  for (int t = 0; t <= k; ++t) {
    const int64_t r0 = (t > 0) ? t - 1 : 0;  // first row touched at this step
    if (t > 0) {
      // ---- pivot of step t-1: the waves' candidates, merged in wave order
      Cand best = cand_empty();
      for (int wv = 0; wv < PJ_WAVES; ++wv) best = cand_merge(best, red[wv]);
      const double nu1 = uniform_f64(best.v1);
      jstar = uniform_i64(best.i1);
      if (t == 1) nu0 = nu1;
      const bool fail = !(nu1 > 0.0) || nu1 <= jb.rank_tol * nu0;
      if (tid == 0) {
        jb.J[t - 1] = jstar;
        if (fail) *jb.status = RID_ERR_RANK;
      }
      if (fail) return;  // the same decision in every thread
      // ---- reflector of step t-1 from the pivot column as the previous
      // step left it (stored before the barrier that ended that step)
      if (wave == 0) make_reflector<RR>(Y + jstar * ldy, r0, l, lane, v_s, tau_s, beta_s);
      __syncthreads();
    }
    const double2 tau = (t > 0) ? tau_s : make_double2(0.0, 0.0);
    const double beta = (t > 0) ? beta_s : 0.0;
    const int nbytes = static_cast<int>((l - r0) * 16);
    const int lo = lane * 16;
    Cand wc = cand_empty();
    for (int64_t c0 = int64_t(wave) * CB; c0 < n; c0 += int64_t(PJ_WAVES) * CB) {
      double2 y[CB][RR];
      __amdgpu_buffer_rsrc_t rs[CB];
      bool live[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int64_t j = c0 + b;
        const bool open_j = j < n && mark[j < n ? j : 0] < 0;
        if (open_j && j == jstar) {
          // the pivot of step t-1: beta at row r0, zeros below
          const __amdgpu_buffer_rsrc_t rp = buf_rsrc(Y + j * ldy + r0, nbytes);
#pragma unroll
          for (int h = 0; h < RR; ++h)
            buf_st(rp, lo + 1024 * h,
                   (h == 0 && lane == 0) ? make_double2(beta, 0.0) : make_double2(0.0, 0.0));
          if (lane == 0) mark[j] = t - 1;
        }
        live[b] = open_j && j != jstar;
        rs[b] = buf_rsrc(live[b] ? Y + j * ldy + r0 : Y, live[b] ? nbytes : 0);
#pragma unroll
        for (int h = 0; h < RR; ++h) y[b][h] = buf_ld(rs[b], lo + 1024 * h);
      }
      if (t > 0) {
        apply_reflector<RR, CB>(y, v_s, tau, lane, 0u);
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int h = 0; h < RR; ++h) buf_st(rs[b], lo + 1024 * h, y[b][h]);
      }
      if (t < k) {
        // rows t .. l-1: all but row r0 = t-1 (lane 0 of slot 0) when t > 0
        const bool below = lane >= t - r0;
        double ss[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) ss[b] = rows_norm2<RR>(y[b], below);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
          const double nrm = sqrt(wave_sum(ss[b]));
          if (live[b]) wc = cand_merge(wc, Cand{nrm, c0 + b, -1.0, wave});
        }
      }
    }
    if (t >= k) return;
    if (lane == 0) red[wave] = wc;
    __syncthreads();  // candidates in LDS; every column of this step stored
  }
}

// Block b runs the whole QR of job order[b] (a batch's rows in play are at
// most 224, so 1 to 4 rows per lane).
__global__ __launch_bounds__(64 * PJ_WAVES) void pivqr_job_kernel(
    const PivJob *__restrict__ jobs, const int *__restrict__ order) {
  __shared__ double2 v_s[64 * 4];
  __shared__ Cand red[PJ_WAVES];
  __shared__ double2 tau_s;
  __shared__ double beta_s;
  const PivJob &jb = jobs[order[blockIdx.x]];
  switch ((jb.l + 63) / 64) {
    case 1: pivqr_job_body<1, 4>(jb, v_s, red, tau_s, beta_s); break;
    case 2: pivqr_job_body<2, 4>(jb, v_s, red, tau_s, beta_s); break;
    case 3: pivqr_job_body<3, 4>(jb, v_s, red, tau_s, beta_s); break;
    case 4: pivqr_job_body<4, 4>(jb, v_s, red, tau_s, beta_s); break;
    default: break;
  }
}

// ---------------------------------------------------------------- CGS2
// The paper's QR method (Sec. 3.2): Gram-Schmidt with reorthogonalisation,
// here right-looking with the same exact pivoting as the Householder steps.
// Y holds the residual columns r_j = (I - Q Q^H) y_j of the unpicked
// columns, updated in place (r_j -= q_t (q_t^H r_j), R(t, j) = q_t^H r_j),
// so the trailing norms |r_j| are exact.  The new direction q_t comes from
// the pivot's residual column reorthogonalised once more against q_0 ..
// q_{t-1} (the second pass of CGS2) and normalised; R(t, j*) = its norm.
// R (k x n, zero below the picked rows) is kept in the workspace and copied
// into Y(0:k, :) after the last step.  Step t is two launches: the pick
// kernel (one workgroup) merges the candidates of step t-1, forms q_{t-1}
// once and stores it with the pivot; the apply kernel (one workgroup per
// 64 columns) applies it and publishes the candidates of step t (parity
// buffers, full residual columns).

template <int RR>
__global__ __launch_bounds__(256) void cgs2_pick_kernel(int t, int64_t l, int64_t n, int64_t k,
                                                        int64_t *perm, double *gaps,
                                                        double rank_tol, PivWs w, double2 *Q,
                                                        double2 *Rk, int *status, int64_t nb) {
  constexpr int QU = 4;                    // directions per wave in flight
  __shared__ double2 vs[64 * RR];          // the pivot's residual column, then v
  __shared__ double2 c_s[1024];            // c_i = q_i^H v
  __shared__ Cand red[4];
  __shared__ double part[256];
  __shared__ int status_s;
  if (threadIdx.x == 0) status_s = *status;
  __syncthreads();
  if (status_s != RID_OK) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t rd = ((t - 1) & 1) * nb;
  Cand cd = cand_empty();
  for (int64_t b = tid; b < nb; b += 256) {
    Cand x{w.cnorm[rd + b], w.cidx[rd + b], w.cnorm2[rd + b], 0};
    if (x.v1 < 0.0) x = cand_empty();
    cd = cand_merge(cd, x);
  }
  const Cand best = cand_block_merge(cd, red);
  const double nu1 = best.v1;
  const double nu0 = (t == 1) ? nu1 : *w.nu0;
  const bool fail = !(nu1 > 0.0) || nu1 <= rank_tol * nu0;
  if (tid == 0) {
    perm[t - 1] = best.i1;
    if (gaps) gaps[t - 1] = (best.v2 < 0.0) ? 1.0 : (nu1 - best.v2) / nu1;
    if (t == 1) *w.nu0 = nu1;
    if (fail) *status = RID_ERR_RANK;
  }
  if (fail) return;
  const int64_t jstar = best.i1;
  const double2 *x = w.ccol + (rd + jstar / PQ_COLS) * l;
  for (int idx = tid; idx < 64 * RR; idx += 256)
    vs[idx] = (idx < l) ? x[idx] : make_double2(0.0, 0.0);
  __syncthreads();
  // second Gram-Schmidt pass, coefficients: wave w takes directions
  // i = w QU + 4 QU u + e (e < QU), QU dot products at a time
  const int64_t nq = t - 1;
  for (int64_t i0 = int64_t(wave) * QU; i0 < nq; i0 += 4 * QU) {
    double dr[QU], di[QU];
#pragma unroll
    for (int e = 0; e < QU; ++e) dr[e] = di[e] = 0.0;
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t row = lane + 64 * h;
      if (row >= l) break;
      const double2 vv = vs[row];
#pragma unroll
      for (int e = 0; e < QU; ++e) {
        if (i0 + e < nq) {
          const double2 qv = Q[(i0 + e) * l + row];
          dr[e] += qv.x * vv.x + qv.y * vv.y;
          di[e] += qv.x * vv.y - qv.y * vv.x;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < QU; ++e) {
      const double a = wave_sum(dr[e]), b = wave_sum(di[e]);
      if (lane == 0 && i0 + e < nq) c_s[i0 + e] = make_double2(a, b);
    }
  }
  __syncthreads();
  // v -= sum_i c_i q_i: threads over rows, QU directions per iteration
  double ss = 0.0;
  for (int64_t row = tid; row < l; row += 256) {
    double2 acc = vs[row];
    for (int64_t i = 0; i < nq; i += QU) {
#pragma unroll
      for (int e = 0; e < QU; ++e) {
        if (i + e < nq) {
          const double2 c = c_s[i + e];
          const double2 qv = Q[(i + e) * l + row];
          acc.x -= qv.x * c.x - qv.y * c.y;
          acc.y -= qv.x * c.y + qv.y * c.x;
        }
      }
    }
    vs[row] = acc;
    ss += acc.x * acc.x + acc.y * acc.y;
  }
  part[tid] = ss;
  __syncthreads();
  for (int st = 128; st >= 1; st >>= 1) {
    if (tid < st) part[tid] += part[tid + st];
    __syncthreads();
  }
  const double nrm = sqrt(part[0]);
  for (int64_t row = tid; row < l; row += 256)
    Q[(t - 1) * l + row] = make_double2(vs[row].x / nrm, vs[row].y / nrm);
  if (tid == 0) {
    Rk[jstar * k + (t - 1)] = make_double2(nrm, 0.0);
    w.pstep[jstar] = t - 1;
  }
}

// The second pass of a step with many earlier directions, spread over the
// device (one workgroup reads every earlier direction twice per step, which
// at k = 1000 costs more than the rest of the QR):
//   head   (1 workgroup)  merge, pivot, copy of the pivot's residual into v;
//   coef   (16 directions per workgroup)  c_i = q_i^H v, each by one wave
//          exactly as in the one-workgroup pick;
//   update (256 rows x CG_DCH directions per workgroup)  chunk 0 starts from
//          v and subtracts its c_i q_i in order, later chunks accumulate theirs
//          from zero;
//   finish (1 workgroup)  v' = chunk 0 - chunk 1 - ... in order, norm,
//          q_{t-1} = v' / |v'|, R(t-1, j*).
// With one chunk the arithmetic is that of the one-workgroup pick, term by
// term; with more, only the association of the row sums differs.
constexpr int CG_SPLIT = 64;    // earlier directions above which the pass is spread
constexpr int CG_DCH = 128;     // directions per update chunk

struct CgsSplit {
  double2 *v;      // [l] the pivot's residual
  double2 *c;      // [k] coefficients of the second pass
  double2 *part;   // [ceil(k / CG_DCH)][l] row sums per chunk
  int64_t *jst;    // [1] the pivot of the step
};

template <int RR>
__global__ __launch_bounds__(256) void cgs2_head_kernel(int t, int64_t l, int64_t *perm,
                                                        double *gaps, double rank_tol, PivWs w,
                                                        CgsSplit cs, int *status, int64_t nb) {
  __shared__ Cand red[4];
  __shared__ int status_s;
  if (threadIdx.x == 0) status_s = *status;
  __syncthreads();
  if (status_s != RID_OK) return;
  const int tid = threadIdx.x;
  const int64_t rd = ((t - 1) & 1) * nb;
  Cand cd = cand_empty();
  for (int64_t b = tid; b < nb; b += 256) {
    Cand x{w.cnorm[rd + b], w.cidx[rd + b], w.cnorm2[rd + b], 0};
    if (x.v1 < 0.0) x = cand_empty();
    cd = cand_merge(cd, x);
  }
  const Cand best = cand_block_merge(cd, red);
  const double nu1 = best.v1;
  const double nu0 = (t == 1) ? nu1 : *w.nu0;
  const bool fail = !(nu1 > 0.0) || nu1 <= rank_tol * nu0;
  if (tid == 0) {
    perm[t - 1] = best.i1;
    if (gaps) gaps[t - 1] = (best.v2 < 0.0) ? 1.0 : (nu1 - best.v2) / nu1;
    if (t == 1) *w.nu0 = nu1;
    if (fail) *status = RID_ERR_RANK;
    else *cs.jst = best.i1;
  }
  if (fail) return;
  const double2 *x = w.ccol + (rd + best.i1 / PQ_COLS) * l;
  for (int64_t row = tid; row < l; row += 256) cs.v[row] = x[row];
}

template <int RR>
__global__ __launch_bounds__(256) void cgs2_coef_kernel(int t, int64_t l, const double2 *Q,
                                                        CgsSplit cs, const int *status) {
  constexpr int QU = 4;
  __shared__ double2 vs[64 * RR];
  __shared__ int status_s;
  if (threadIdx.x == 0) status_s = *status;
  __syncthreads();
  if (status_s != RID_OK) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  for (int idx = tid; idx < 64 * RR; idx += 256)
    vs[idx] = (idx < l) ? cs.v[idx] : make_double2(0.0, 0.0);
  __syncthreads();
  const int64_t nq = t - 1;
  const int64_t i0 = int64_t(blockIdx.x) * 16 + wave * QU;
  if (i0 >= nq) return;
  double dr[QU], di[QU];
#pragma unroll
  for (int e = 0; e < QU; ++e) dr[e] = di[e] = 0.0;
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const int64_t row = lane + 64 * h;
    if (row >= l) break;
    const double2 vv = vs[row];
#pragma unroll
    for (int e = 0; e < QU; ++e) {
      if (i0 + e < nq) {
        const double2 qv = Q[(i0 + e) * l + row];
        dr[e] += qv.x * vv.x + qv.y * vv.y;
        di[e] += qv.x * vv.y - qv.y * vv.x;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < QU; ++e) {
    const double a = wave_sum(dr[e]), b = wave_sum(di[e]);
    if (lane == 0 && i0 + e < nq) cs.c[i0 + e] = make_double2(a, b);
  }
}

// grid (row blocks of 256, direction chunks of CG_DCH)
__global__ __launch_bounds__(256) void cgs2_update_kernel(int t, int64_t l, const double2 *Q,
                                                          CgsSplit cs, const int *status) {
  constexpr int QU = 4;
  if (*status != RID_OK) return;
  const int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (row >= l) return;
  const int64_t nq = t - 1;
  const int64_t dc = blockIdx.y;
  const int64_t ib = dc * CG_DCH;
  const int64_t ie = min(nq, ib + CG_DCH);
  double2 acc;
  if (dc == 0) {
    acc = cs.v[row];
    for (int64_t i = ib; i < ie; i += QU) {
#pragma unroll
      for (int e = 0; e < QU; ++e) {
        if (i + e < ie) {
          const double2 c = cs.c[i + e];
          const double2 qv = Q[(i + e) * l + row];
          acc.x -= qv.x * c.x - qv.y * c.y;
          acc.y -= qv.x * c.y + qv.y * c.x;
        }
      }
    }
  } else {
    acc = make_double2(0.0, 0.0);
    for (int64_t i = ib; i < ie; i += QU) {
#pragma unroll
      for (int e = 0; e < QU; ++e) {
        if (i + e < ie) {
          const double2 c = cs.c[i + e];
          const double2 qv = Q[(i + e) * l + row];
          acc.x += qv.x * c.x - qv.y * c.y;
          acc.y += qv.x * c.y + qv.y * c.x;
        }
      }
    }
  }
  cs.part[dc * l + row] = acc;
}

template <int RR>
__global__ __launch_bounds__(256) void cgs2_finish_kernel(int t, int64_t l, int64_t k, int ndc,
                                                          PivWs w, CgsSplit cs, double2 *Q,
                                                          double2 *Rk, const int *status) {
  __shared__ double2 vs[64 * RR];
  __shared__ double part[256];
  __shared__ int status_s;
  if (threadIdx.x == 0) status_s = *status;
  __syncthreads();
  if (status_s != RID_OK) return;
  const int tid = threadIdx.x;
  double ss = 0.0;
  for (int64_t row = tid; row < l; row += 256) {
    double2 acc = cs.part[row];
    for (int dc = 1; dc < ndc; ++dc) {
      const double2 p = cs.part[dc * l + row];
      acc.x -= p.x;
      acc.y -= p.y;
    }
    vs[row] = acc;
    ss += acc.x * acc.x + acc.y * acc.y;
  }
  part[tid] = ss;
  __syncthreads();
  for (int st = 128; st >= 1; st >>= 1) {
    if (tid < st) part[tid] += part[tid + st];
    __syncthreads();
  }
  const double nrm = sqrt(part[0]);
  for (int64_t row = tid; row < l; row += 256)
    Q[(t - 1) * l + row] = make_double2(vs[row].x / nrm, vs[row].y / nrm);
  if (tid == 0) {
    const int64_t jstar = *cs.jst;
    Rk[jstar * k + (t - 1)] = make_double2(nrm, 0.0);
    w.pstep[jstar] = t - 1;
  }
}

template <int RR>
__global__ __launch_bounds__(256) void cgs2_apply_kernel(int t, int64_t l, int64_t n, int64_t k,
                                                         double2 *Y, int64_t ldy, PivWs w,
                                                         const double2 *Q, double2 *Rk,
                                                         int *status) {
  __shared__ double2 q_s[64 * RR];
  __shared__ Cand red[4];
  __shared__ int status_s;
  if (threadIdx.x == 0) status_s = *status;
  __syncthreads();
  if (status_s != RID_OK) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // uniform in the wave; read as such, so that buffer resources built from
  // it stay in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t bx = blockIdx.x;
  const int64_t nb = gridDim.x;
  const int64_t cbeg = bx * PQ_COLS;
  const int64_t wr = (t & 1) * nb;
  if (t > 0) {
    for (int idx = tid; idx < 64 * RR; idx += 256)
      q_s[idx] = (idx < l) ? Q[(t - 1) * l + idx] : make_double2(0.0, 0.0);
    __syncthreads();
  }
  // A column is rows 0 .. l-1 through a range-checked buffer resource: rows
  // past l load as zeros (as q holds there) and are never stored.  The
  // picked-step marks of the wave's 16 columns are read at once (bit c set:
  // unpicked; the pivot of this step is already marked).
  const int64_t jw = cbeg + wave * 16;
  const bool inr = lane < 16 && jw + lane < n;
  const uint64_t open = __ballot(inr && w.pstep[inr ? jw + lane : 0] < 0);
  const int nbytes = static_cast<int>(l * 16);
  const int lo = lane * 16;
  Cand wc = cand_empty();
  for (int cc = 0; cc < 16; ++cc) {
    if (!((open >> cc) & 1)) continue;
    const int64_t j = jw + cc;
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(Y + j * ldy, nbytes);
    double2 y[RR];
#pragma unroll
    for (int h = 0; h < RR; ++h) y[h] = buf_ld(rs, lo + 1024 * h);
    if (t > 0) {
      // r = q^H y, then y -= q r, as FMA chains
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int h = 0; h < RR; ++h) {
        const double2 qv = q_s[lane + 64 * h];
        dr = fma(qv.x, y[h].x, dr);
        dr = fma(qv.y, y[h].y, dr);
        di = fma(qv.x, y[h].y, di);
        di = fma(-qv.y, y[h].x, di);
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      if (lane == 0) Rk[j * k + (t - 1)] = make_double2(dr, di);
#pragma unroll
      for (int h = 0; h < RR; ++h) {
        const double2 qv = q_s[lane + 64 * h];
        y[h].x = fma(-qv.x, dr, y[h].x);
        y[h].x = fma(qv.y, di, y[h].x);
        y[h].y = fma(-qv.x, di, y[h].y);
        y[h].y = fma(-qv.y, dr, y[h].y);
        buf_st(rs, lo + 1024 * h, y[h]);
      }
    }
    if (t < k) {
      double ss = 0.0;
#pragma unroll
      for (int h = 0; h < RR; ++h) {
        ss = fma(y[h].x, y[h].x, ss);
        ss = fma(y[h].y, y[h].y, ss);
      }
      wc = cand_merge(wc, Cand{sqrt(wave_sum(ss)), j, -1.0, wave});
    }
  }
  if (t >= k) return;
  if (lane == 0) red[wave] = wc;
  __syncthreads();
  Cand bc = cand_empty();
  for (int wv = 0; wv < 4; ++wv) bc = cand_merge(bc, red[wv]);
  if (tid == 0) {
    w.cnorm[wr + bx] = bc.v1;
    w.cnorm2[wr + bx] = bc.v2;
    w.cidx[wr + bx] = bc.i1;
  }
  if (bc.src >= 0) {
    const double2 *src = Y + bc.i1 * ldy;
    double2 *dst = w.ccol + (wr + bx) * l;
    for (int64_t row = tid; row < l; row += 256) dst[row] = src[row];
  }
}

__global__ void cgs2_zero_kernel(int64_t count, double2 *p) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < count;
       e += int64_t(gridDim.x) * blockDim.x)
    p[e] = make_double2(0.0, 0.0);
}

// Y(0:k, j) = R(:, j) once every step is done.
__global__ void cgs2_copy_r_kernel(int64_t n, int64_t k, const double2 *__restrict__ Rk,
                                   double2 *__restrict__ Y, int64_t ldy, const int *status) {
  if (*status != RID_OK) return;
  const int64_t total = n * k;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = e / k;
    Y[j * ldy + (e - j * k)] = Rk[e];
  }
}

// perm[k + r] = r-th unpicked column in increasing order (one workgroup).
__global__ __launch_bounds__(1024) void pivqr_tail_kernel(int64_t n, int64_t k,
                                                          const int *pstep, int64_t *perm,
                                                          const int *status) {
  __shared__ int wcount[16];
  if (*status != RID_OK) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int64_t base = k;
  for (int64_t c0 = 0; c0 < n; c0 += 1024) {
    const int64_t j = c0 + tid;
    const bool flag = (j < n) && pstep[j] < 0;
    const uint64_t mask = __ballot(flag);
    const int before = __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wcount[wave] = __popcll(mask);
    __syncthreads();
    int off = 0, total = 0;
    for (int wv = 0; wv < 16; ++wv) {
      if (wv < wave) off += wcount[wv];
      total += wcount[wv];
    }
    if (flag) perm[base + off + before] = j;
    base += total;
    __syncthreads();
  }
}

// rows per lane for l rows in play: the smallest of 1, 2, 3, 4, 6, 8, 12, 16,
// 24, 32 with 64 RR >= l (0 when l > 2048)
int pick_rr(int64_t l) {
  static const int opts[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
  for (int o : opts)
    if (64 * o >= l) return o;
  return 0;
}

// The panel form's steps run at one wave per SIMD from 16 rows per lane up,
// so it also takes 20 and 28 rows per lane: fewer registers and
// instructions on rows past l.
int pick_rr_panel(int64_t l) {
  static const int opts[] = {1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 28, 32};
  for (int o : opts)
    if (64 * o >= l) return o;
  return 0;
}

template <class F>
void with_rr(int rr, F &&f) {
  switch (rr) {
    case 1: f(std::integral_constant<int, 1>()); break;
    case 2: f(std::integral_constant<int, 2>()); break;
    case 3: f(std::integral_constant<int, 3>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 6: f(std::integral_constant<int, 6>()); break;
    case 8: f(std::integral_constant<int, 8>()); break;
    case 12: f(std::integral_constant<int, 12>()); break;
    case 16: f(std::integral_constant<int, 16>()); break;
    case 20: f(std::integral_constant<int, 20>()); break;
    case 24: f(std::integral_constant<int, 24>()); break;
    case 28: f(std::integral_constant<int, 28>()); break;
    case 32: f(std::integral_constant<int, 32>()); break;
    default: break;
  }
}

// Step t touches rows t-1 .. l-1 only, so each launch takes the smallest RR
// that covers them: at l = 2k the rows in play halve over the QR.
void launch_steps(hipStream_t st, int64_t l, int64_t n, int64_t k, double2 *Y, int64_t ldy,
                  int64_t *perm, double *gaps, double rank_tol, const PivWs &w, int *status) {
  const unsigned nb = static_cast<unsigned>((n + PQ_COLS - 1) / PQ_COLS);
  // With few workgroups per step (n / 64 <= 512: at most two waves per
  // SIMD) each wave is a chain of dependent loads and reductions, and taking
  // several columns at a time gains more than the occupancy it costs; with
  // more workgroups the occupancy wins (200 x 2^16: 5.9 ms one at a time,
  // 7.3 ms four at a time).
  const bool wide = nb <= 512;
  for (int t = 0; t <= k; ++t) {
    const int64_t r0 = (t > 0) ? t - 1 : 0;
    with_rr(pick_rr(l - r0), [&](auto R) {
      constexpr int RR = decltype(R)::value;
      constexpr int CBW = RR <= 4 ? 4 : (RR <= 8 ? 2 : 1);
      if (wide)
        hipLaunchKernelGGL((pivqr_step_kernel<RR, CBW>), dim3(nb), dim3(256), 0, st, t, l, n, k,
                           Y, ldy, perm, gaps, rank_tol, w, status);
      else
        hipLaunchKernelGGL((pivqr_step_kernel<RR, 1>), dim3(nb), dim3(256), 0, st, t, l, n, k, Y,
                           ldy, perm, gaps, rank_tol, w, status);
    });
  }
}

// The panel form for a Y that does not fit the last-level cache; the
// environment variable RID_QR_PANEL=1 (=0) forces (forbids) it, and
// RID_QR_PANEL_GROUPS caps its workgroups per step.
bool pivqr_panel_wanted(int64_t l, int64_t n) {
  const char *e = std::getenv("RID_QR_PANEL");
  if (e && e[0] == '1') return true;
  if (e && e[0] == '0') return false;
  return double(l) * double(n) * 16.0 > 512.0 * 1024 * 1024;
}

// rows a .. l-1 are in play at step t; RR is picked per launch as above
// Workgroups of the panel kernel at RR that the device holds at once (its
// occupancy times the compute units), found once per RR and device.
template <int RR>
int64_t panel_resident() {
  static int64_t cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cached[dev] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&pivqr_panel_kernel<RR, 1>), 256, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    cached[dev] = int64_t(per_cu > 0 ? per_cu : 1) * int64_t(cus > 0 ? cus : 1);
  }
  return cached[dev];
}

void launch_panel_steps(hipStream_t st, int64_t l, int64_t n, int64_t k, double2 *Y,
                        int64_t ldy, int64_t *perm, double *gaps, double rank_tol,
                        const PivWs &w, const PanelWs &pw, int *status) {
  const int64_t nbk = (n + PQ_COLS - 1) / PQ_COLS;
  // RID_QR_PANEL_GROUPS=g caps the workgroups per step (each then takes more
  // column blocks); the results do not depend on it
  const char *ge = std::getenv("RID_QR_PANEL_GROUPS");
  const int64_t groups_cap = ge ? std::atoll(ge) : 0;
  int a = 0;          // first reflector not yet written into Y
  int64_t gprev = 0;  // candidate slots of the previous step
  for (int t = 0; t <= k; ++t) {
    const int wr = (t > 0 && (t - a >= QP_NB || t == k)) ? 1 : 0;
    with_rr(pick_rr_panel(l - a), [&](auto R) {
      constexpr int RR = decltype(R)::value;
      // as many workgroups as fit at once (each loops over column blocks),
      // never more than there are blocks
      const int64_t res = panel_resident<RR>();
      int64_t g = (res > 0 && res < nbk) ? res : nbk;
      if (groups_cap > 0 && groups_cap < g) g = groups_cap;
      // one column at a time: two (CB = 2) gained under 2% at RR = 24 and
      // lost at RR <= 16, where their registers cost occupancy
      hipLaunchKernelGGL((pivqr_panel_kernel<RR, 1>), dim3(static_cast<unsigned>(g)), dim3(256),
                         0, st, t, a, wr, l, n, k, Y, ldy, perm, gaps, rank_tol, w, pw, status,
                         nbk, gprev);
      gprev = g;
    });
    if (wr) a = t;
  }
}

}  // namespace

bool pivqr_supported(int64_t l) { return l >= 1 && pick_rr(l) > 0; }

size_t pivqr_ws_bytes(int64_t l, int64_t n, int64_t k, int kind) {
  size_t b = piv_bytes(l, n);
  {
    WsCarve c(nullptr);  // panel reflector slots
    c.take<double2>(size_t(QP_NB) * size_t(l));
    c.take<double2>(QP_NB);
    b += c.off + 256;
  }
  if (kind == RID_QR_CGS2) {
    WsCarve c(nullptr);
    c.take<double2>(size_t(l) * size_t(k));
    c.take<double2>(size_t(k) * size_t(n));
    c.take<double2>(size_t(l));
    c.take<double2>(size_t(k > 0 ? k : 1));
    c.take<double2>(size_t((k + CG_DCH - 1) / CG_DCH + 1) * size_t(l));
    c.take<int64_t>(1);
    b += c.off + 256;
  }
  return b;
}

int64_t pivqr_blocks(int64_t n) { return (n + PQ_COLS - 1) / PQ_COLS; }

size_t pivqr_job_ws_bytes(int64_t l, int64_t n) {
  WsCarve c(nullptr);
  const int64_t nb = pivqr_blocks(n);
  c.take<double>(2 * nb);
  c.take<double>(2 * nb);
  c.take<int64_t>(2 * nb);
  c.take<double2>(2 * size_t(nb) * size_t(l));
  c.take<double>(1);
  return c.off;
}

void pivqr_job_carve(char *base, PivJob &jb) {
  WsCarve c(base);
  const int64_t nb = pivqr_blocks(jb.n);
  jb.cnorm = c.take<double>(2 * nb);
  jb.cnorm2 = c.take<double>(2 * nb);
  jb.cidx = c.take<int64_t>(2 * nb);
  jb.ccol = c.take<double2>(2 * size_t(nb) * size_t(jb.l));
  jb.nu0 = c.take<double>(1);
}

hipError_t launch_pivqr_batch(hipStream_t st, const int64_t *lmax, const int64_t *live,
                              int64_t kmax, const PivJob *djobs, const int4 *dtab, int64_t count,
                              RidProf *prof, int cb) {
  if (count == 0) return hipSuccess;
  ProfScope ps(prof, st, RID_KERNEL_PIVQR);
  hipLaunchKernelGGL(pivqr_init_grouped, dim3(static_cast<unsigned>(count)), dim3(256), 0, st,
                     djobs, dtab);
  for (int t = 0; t <= kmax; ++t) {
    const int64_t nlive = std::min(live[t], count);
    if (nlive <= 0) continue;
    const dim3 grid(static_cast<unsigned>(nlive));
    // the live jobs' rows in play, t-1 .. l-1, fit in lmax[t] - (t-1)
    with_rr(pick_rr(lmax[t] - (t > 0 ? t - 1 : 0)), [&](auto R) {
      constexpr int RR = decltype(R)::value;
      if constexpr (RR <= 4) {
        if (cb == 4)
          hipLaunchKernelGGL((pivqr_step_grouped<RR, 4>), grid, dim3(256), 0, st, t, djobs, dtab);
        else if (cb == 2)
          hipLaunchKernelGGL((pivqr_step_grouped<RR, 2>), grid, dim3(256), 0, st, t, djobs, dtab);
        else
          hipLaunchKernelGGL((pivqr_step_grouped<RR, 1>), grid, dim3(256), 0, st, t, djobs, dtab);
      }
    });
  }
  ps.stop();
  return hipGetLastError();
}

hipError_t launch_pivqr_jobs(hipStream_t st, const PivJob *djobs, const int *dorder, int count,
                             RidProf *prof) {
  if (count == 0) return hipSuccess;
  ProfScope ps(prof, st, RID_KERNEL_PIVQR);
  hipLaunchKernelGGL(pivqr_job_kernel, dim3(static_cast<unsigned>(count)), dim3(64 * PJ_WAVES), 0,
                     st, djobs, dorder);
  ps.stop();
  return hipGetLastError();
}

hipError_t launch_pivqr(hipStream_t st, int64_t l, int64_t n, int64_t k, double2 *Y,
                        int64_t ldy, int64_t *perm, double *gaps, double rank_tol, void *ws,
                        int *d_status, RidProf *prof, int kind) {
  const PivWs w = carve_piv(ws, l, n);
  ProfScope ps(prof, st, RID_KERNEL_PIVQR);
  hipLaunchKernelGGL(pivqr_init_kernel, dim3(static_cast<unsigned>((n + 255) / 256)),
                     dim3(256), 0, st, n, w.pstep, d_status);
  if (kind == RID_QR_CGS2) {
    WsCarve c(static_cast<char *>(ws) + piv_bytes(l, n));
    double2 *Q = c.take<double2>(size_t(l) * size_t(k));
    double2 *Rk = c.take<double2>(size_t(k) * size_t(n));
    CgsSplit cs;
    cs.v = c.take<double2>(size_t(l));
    cs.c = c.take<double2>(size_t(k > 0 ? k : 1));
    cs.part = c.take<double2>(size_t((k + CG_DCH - 1) / CG_DCH + 1) * size_t(l));
    cs.jst = c.take<int64_t>(1);
    const int64_t rcount = k * n;
    hipLaunchKernelGGL(cgs2_zero_kernel,
                       dim3(static_cast<unsigned>(std::min<int64_t>((rcount + 255) / 256, 65536))),
                       dim3(256), 0, st, rcount, Rk);
    const unsigned nb = static_cast<unsigned>((n + PQ_COLS - 1) / PQ_COLS);
    with_rr(pick_rr(l), [&](auto R) {
      constexpr int RR = decltype(R)::value;
      for (int t = 0; t <= k; ++t) {
        const int64_t nq = t - 1;  // earlier directions of the second pass
        if (t > 0 && nq <= CG_SPLIT) {
          hipLaunchKernelGGL(cgs2_pick_kernel<RR>, dim3(1), dim3(256), 0, st, t, l, n, k, perm,
                             gaps, rank_tol, w, Q, Rk, d_status, int64_t(nb));
        } else if (t > 0) {
          const int ndc = static_cast<int>((nq + CG_DCH - 1) / CG_DCH);
          hipLaunchKernelGGL(cgs2_head_kernel<RR>, dim3(1), dim3(256), 0, st, t, l, perm, gaps,
                             rank_tol, w, cs, d_status, int64_t(nb));
          hipLaunchKernelGGL(cgs2_coef_kernel<RR>, dim3(static_cast<unsigned>((nq + 15) / 16)),
                             dim3(256), 0, st, t, l, Q, cs, d_status);
          hipLaunchKernelGGL(cgs2_update_kernel,
                             dim3(static_cast<unsigned>((l + 255) / 256), static_cast<unsigned>(ndc)),
                             dim3(256), 0, st, t, l, Q, cs, d_status);
          hipLaunchKernelGGL(cgs2_finish_kernel<RR>, dim3(1), dim3(256), 0, st, t, l, k, ndc, w,
                             cs, Q, Rk, d_status);
        }
        hipLaunchKernelGGL(cgs2_apply_kernel<RR>, dim3(nb), dim3(256), 0, st, t, l, n, k, Y, ldy,
                           w, Q, Rk, d_status);
      }
    });
    hipLaunchKernelGGL(cgs2_copy_r_kernel,
                       dim3(static_cast<unsigned>(std::min<int64_t>((rcount + 255) / 256, 65536))),
                       dim3(256), 0, st, n, k, Rk, Y, ldy, d_status);
  } else if (pivqr_panel_wanted(l, n)) {
    WsCarve c(static_cast<char *>(ws) + piv_bytes(l, n));
    PanelWs pw;
    pw.V = c.take<double2>(size_t(QP_NB) * size_t(l));
    pw.tau = c.take<double2>(QP_NB);
    launch_panel_steps(st, l, n, k, Y, ldy, perm, gaps, rank_tol, w, pw, d_status);
  } else {
    launch_steps(st, l, n, k, Y, ldy, perm, gaps, rank_tol, w, d_status);
  }
  hipLaunchKernelGGL(pivqr_tail_kernel, dim3(1), dim3(1024), 0, st, n, k, w.pstep, perm,
                     d_status);
  ps.stop();
  return hipGetLastError();
}
