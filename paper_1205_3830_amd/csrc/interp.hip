// interp.hip -- the interpolation matrix of Sec. 2: solve R2 = R1 T by back
// substitution, each column on its own (the column-parallel "factorization
// of R" of Sec. 3.2), and write P = [I T] in the original column order.
//
// k <= 256: four columns of P per wave.  The k right-hand-side entries of
// a column sit in the lanes (RR per lane, k <= 64 RR); step t multiplies
// entry t by the reciprocal of the diagonal R1(t, t) and updates the
// entries above it with column t of R1 (= column J[t] of R, a coalesced
// read that the wave's columns share, and all columns through the L2).
// The reads of the next steps are in flight during the arithmetic of step
// t.  Larger k (up to 1024), where k dependent steps
// per column would leave the device latency-bound: R1^-1 once (k columns),
// then P = R1^-1 R(0:k, :) as one GEMM on the FP64 matrix cores.
#include "rid_internal.hpp"

namespace {

constexpr int INTERP_CPW = 4;  // columns of P per wave of the direct solve

__global__ void interp_mark_clear_kernel(int64_t n, int *mark) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j < n) mark[j] = -1;
}

__global__ void interp_mark_set_kernel(int64_t n, int64_t k, const int64_t *J, int *mark) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t < k) {
    const int64_t j = J[t];
    if (j >= 0 && j < n) mark[j] = static_cast<int>(t);
  }
}

// Steps of R1 columns loaded ahead of their use (a ring of registers).
template <int RR>
constexpr int interp_depth() {
  return RR == 1 ? 8 : (RR == 2 ? 4 : 2);
}

// Rows 0 .. t-1 of column t of R1 (column J[t] of R) into the lanes, zeros
// from row t on (the buffer's range check); all zeros for t <= 0.  Lane s
// holds J[s + 64 h] in js[h]; the index is read out of its lane.
template <int RR>
RID_DEV void r1_column(double2 (&dst)[RR], const double2 *R, int64_t ldr,
                       const int64_t (&js)[RR], int64_t t, int lane) {
  const int64_t tc = t > 0 ? t : 0;
  int64_t jv = js[0];
#pragma unroll
  for (int h = 1; h < RR; ++h)
    if (h == static_cast<int>(tc >> 6)) jv = js[h];
  const int src = static_cast<int>(tc & 63);
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(jv), src);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(jv >> 32), src);
  const int64_t jt = static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(R + jt * ldr, t > 0 ? static_cast<int>(t) * 16 : 0);
#pragma unroll
  for (int h = 0; h < RR; ++h) dst[h] = buf_ld(rs, (lane + 64 * h) * 16);
}

// Workgroup bx solves columns 16 bx .. 16 bx + 15 of P, INTERP_CPW per
// wave.  The columns of a wave share each load of an R1 column and each
// reciprocal of a diagonal entry: lane s holds 1 / R1(s, s) (conj(d) / |d|^2,
// formed once per wave), step t reads it and the right-hand-side entry t of
// each column out of lane t into scalar registers, so that the quotient
// x_t = r_t / R1(t, t) is one complex product, and updates the entries
// above t.  The R1 columns of the next steps are in flight meanwhile.
template <int RR>
RID_DEV void interp_body(int64_t n, int64_t k, const double2 *__restrict__ R, int64_t ldr,
                         const int64_t *__restrict__ J, double2 *__restrict__ P, int64_t ldp,
                         const int *__restrict__ mark, int64_t bx) {
  constexpr int C = INTERP_CPW;
  constexpr int D = interp_depth<RR>();
  __shared__ int64_t Js[64 * RR];
  for (int t = threadIdx.x; t < 64 * RR; t += blockDim.x) {
    int64_t jt = (t < k) ? J[t] : 0;
    if (jt < 0 || jt >= n) jt = 0;  // keeps every read inside R; such a P is meaningless
    Js[t] = jt;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t j0 = bx * (4 * C) + wave * C;
  if (j0 >= n) return;
  // column c: solved (mark -1), identity column of step mark (>= 0), or past n
  int tid_c[C];
  double2 r[C][RR];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int64_t j = j0 + c;
    tid_c[c] = (j < n) ? mark[j] : -2;
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t s = lane + 64 * h;
      r[c][h] = (tid_c[c] == -1 && s < k) ? R[s + j * ldr] : make_double2(0.0, 0.0);
    }
  }
  double2 dv[RR];
  int64_t js[RR];
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const int64_t s = lane + 64 * h;
    js[h] = Js[s];
    dv[h] = make_double2(0.0, 0.0);
    if (s < k) {
      const double2 d = R[s + js[h] * ldr];
      const double den = d.x * d.x + d.y * d.y;
      dv[h] = make_double2(d.x / den, -d.y / den);
    }
  }
  // the ring, oldest load first (the order that lets the loop wait for one
  // load at a time)
  double2 ring[D][RR];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    r1_column<RR>(ring[d], R, ldr, js, k - 1 - d, lane);
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int64_t tb = k - 1; tb >= 0; tb -= D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      // steps t < 0 of the last round change nothing (every lane's row is
      // at or above 0 > t); running them keeps the loop free of exits
      const int64_t t = tb - d;
      double2 rc[RR];
#pragma unroll
      for (int h = 0; h < RR; ++h) rc[h] = ring[d][h];
      r1_column<RR>(ring[d], R, ldr, js, t - D, lane);
      __builtin_amdgcn_sched_barrier(0);
      const int ht = static_cast<int>(t >> 6);
      const int lt = static_cast<int>(t & 63);
      double2 di = dv[0];
#pragma unroll
      for (int h = 1; h < RR; ++h)
        if (h == ht) di = dv[h];
      const double ix = lane_bcast(di.x, lt), iy = lane_bcast(di.y, lt);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double2 own = r[c][0];
#pragma unroll
        for (int h = 1; h < RR; ++h)
          if (h == ht) own = r[c][h];
        const double ox = lane_bcast(own.x, lt), oy = lane_bcast(own.y, lt);
        const double tx = ox * ix - oy * iy;
        const double ty = ox * iy + oy * ix;
        // row t takes x_t, rows above it the update, rows below keep their
        // final values (selects, not branches)
#pragma unroll
        for (int h = 0; h < RR; ++h) {
          const int64_t s = lane + 64 * h;
          const double ux = r[c][h].x - (rc[h].x * tx - rc[h].y * ty);
          const double uy = r[c][h].y - (rc[h].x * ty + rc[h].y * tx);
          const double2 u = (s < t) ? make_double2(ux, uy) : r[c][h];
          r[c][h] = (s == t) ? make_double2(tx, ty) : u;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if (tid_c[c] == -2) continue;
    double2 *pc = P + (j0 + c) * ldp;
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t s = lane + 64 * h;
      if (s < k)
        pc[s] = (tid_c[c] >= 0) ? make_double2(s == tid_c[c] ? 1.0 : 0.0, 0.0) : r[c][h];
    }
  }
}

template <int RR>
__global__ __launch_bounds__(256) void interp_kernel(int64_t n, int64_t k,
                                                     const double2 *__restrict__ R, int64_t ldr,
                                                     const int64_t *__restrict__ J,
                                                     double2 *__restrict__ P, int64_t ldp,
                                                     const int *__restrict__ mark) {
  interp_body<RR>(n, k, R, ldr, J, P, ldp, mark, blockIdx.x);
}

// A batch: block b solves the columns of group tab[b].y (16 columns) of job
// tab[b].x.
template <int RR>
__global__ __launch_bounds__(256) void interp_kernel_grouped(const InterpJob *__restrict__ jobs,
                                                             const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const InterpJob &jb = jobs[e.x];
  interp_body<RR>(jb.n, jb.k, jb.R, jb.ldr, jb.J, jb.P, jb.ldp, jb.mark, e.y);
}

// Large k (> 256): column c of W = R1^-1 by back substitution of
// R1 w = e_c, one wave per column (w(s) = 0 for s > c, so the steps start
// at t = c); W is stored row-major (entry (s, c) at W[s * ldw + c]) as the
// operator of the GEMM P = W R(0:k, :) that follows.
template <int RR>
__global__ __launch_bounds__(256) void interp_inverse_kernel(int64_t n, int64_t k,
                                                             const double2 *__restrict__ R,
                                                             int64_t ldr,
                                                             const int64_t *__restrict__ J,
                                                             double2 *__restrict__ W,
                                                             int64_t ldw) {
  __shared__ int64_t Js[64 * RR];
  for (int t = threadIdx.x; t < 64 * RR; t += blockDim.x) {
    int64_t jt = (t < k) ? J[t] : 0;
    if (jt < 0 || jt >= n) jt = 0;  // keeps every read inside R; such a W is meaningless
    Js[t] = jt;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t c = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (c >= k) return;
  double2 w[RR];
#pragma unroll
  for (int h = 0; h < RR; ++h)
    w[h] = make_double2((lane + 64 * h == c) ? 1.0 : 0.0, 0.0);
  for (int64_t t = c; t >= 0; --t) {
    const double2 *cj = R + Js[t] * ldr;  // column t of R1
    double2 rc[RR];
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t s = lane + 64 * h;
      rc[h] = (s <= t) ? cj[s] : make_double2(0.0, 0.0);
    }
    const int ht = static_cast<int>(t >> 6);
    const int lt = static_cast<int>(t & 63);
    double2 own = w[0], dg = rc[0];
#pragma unroll
    for (int h = 1; h < RR; ++h)
      if (h == ht) {
        own = w[h];
        dg = rc[h];
      }
    const double ox = lane_bcast(own.x, lt), oy = lane_bcast(own.y, lt);
    const double dx = lane_bcast(dg.x, lt), dy = lane_bcast(dg.y, lt);
    const double den = dx * dx + dy * dy;
    const double tx = (ox * dx + oy * dy) / den;
    const double ty = (oy * dx - ox * dy) / den;
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t s = lane + 64 * h;
      if (s == t) {
        w[h] = make_double2(tx, ty);
      } else if (s < t) {
        w[h].x -= rc[h].x * tx - rc[h].y * ty;
        w[h].y -= rc[h].x * ty + rc[h].y * tx;
      }
    }
  }
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const int64_t s = lane + 64 * h;
    if (s < k) W[s * ldw + c] = w[h];
  }
}

// P(:, J[t]) = e_t exactly (the GEMM gives it only to rounding).
__global__ void interp_identity_kernel(int64_t n, int64_t k, const int64_t *__restrict__ J,
                                       double2 *__restrict__ P, int64_t ldp) {
  const int64_t t = blockIdx.x;
  const int64_t j = J[t];
  if (j < 0 || j >= n) return;
  for (int64_t s = threadIdx.x; s < k; s += blockDim.x)
    P[j * ldp + s] = make_double2(s == t ? 1.0 : 0.0, 0.0);
}

constexpr int64_t INTERP_DIRECT_KMAX = 256;  // per-column solve up to here

}  // namespace

bool interp_supported(int64_t k) { return k >= 1 && k <= 1024; }

int64_t interp_blocks(int64_t n) { return (n + 4 * INTERP_CPW - 1) / (4 * INTERP_CPW); }

size_t interp_ws_bytes(int64_t n, int64_t k) {
  WsCarve c(nullptr);
  c.take<int>(n);
  if (k > INTERP_DIRECT_KMAX) {
    c.take<double2>(size_t(k) * size_t(k));
    c.take<char>(sketch_ws_bytes(RID_C128, RID_FP64, k, n, k));
  }
  return c.off + 256;
}

hipError_t launch_interp(hipStream_t st, int64_t n, int64_t k, const double2 *R, int64_t ldr,
                         const int64_t *J, double2 *P, int64_t ldp, void *ws,
                         RidProf *prof) {
  WsCarve c(ws);
  int *mark = c.take<int>(n);
  if (k > INTERP_DIRECT_KMAX) {
    // T = R1^-1 R2 as W = R1^-1 (k small solves) then P = W R(0:k, :) on the
    // FP64 matrix cores, then P(:, J) = I exactly
    double2 *W = c.take<double2>(size_t(k) * size_t(k));
    void *part = c.take<char>(sketch_ws_bytes(RID_C128, RID_FP64, k, n, k));
    ProfScope ps(prof, st, RID_KERNEL_INTERP);
    const dim3 gw(static_cast<unsigned>((k + 3) / 4));
    if (k <= 512)
      hipLaunchKernelGGL(interp_inverse_kernel<8>, gw, dim3(256), 0, st, n, k, R, ldr, J, W, k);
    else
      hipLaunchKernelGGL(interp_inverse_kernel<16>, gw, dim3(256), 0, st, n, k, R, ldr, J, W, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_sketch(st, RID_C128, RID_FP64, k, n, k, R, ldr, W, k, P, ldp, part, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(interp_identity_kernel, dim3(static_cast<unsigned>(k)), dim3(256), 0, st,
                       n, k, J, P, ldp);
    ps.stop();
    return hipGetLastError();
  }
  const unsigned nbn = static_cast<unsigned>((n + 255) / 256);
  hipLaunchKernelGGL(interp_mark_clear_kernel, dim3(nbn), dim3(256), 0, st, n, mark);
  hipLaunchKernelGGL(interp_mark_set_kernel, dim3(static_cast<unsigned>((k + 255) / 256)),
                     dim3(256), 0, st, n, k, J, mark);
  const unsigned nb = static_cast<unsigned>(interp_blocks(n));
  ProfScope ps(prof, st, RID_KERNEL_INTERP);
  if (k <= 64)
    hipLaunchKernelGGL(interp_kernel<1>, dim3(nb), dim3(256), 0, st, n, k, R, ldr, J, P, ldp,
                       mark);
  else if (k <= 128)
    hipLaunchKernelGGL(interp_kernel<2>, dim3(nb), dim3(256), 0, st, n, k, R, ldr, J, P, ldp,
                       mark);
  else if (k <= 192)
    hipLaunchKernelGGL(interp_kernel<3>, dim3(nb), dim3(256), 0, st, n, k, R, ldr, J, P, ldp,
                       mark);
  else
    hipLaunchKernelGGL(interp_kernel<4>, dim3(nb), dim3(256), 0, st, n, k, R, ldr, J, P, ldp,
                       mark);
  ps.stop();
  return hipGetLastError();
}

hipError_t launch_interp_batch(hipStream_t st, int kmax, const InterpJob *djobs,
                               const int4 *dtab, int64_t count, RidProf *prof) {
  if (count == 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(count));
  ProfScope ps(prof, st, RID_KERNEL_INTERP);
  if (kmax <= 64)
    hipLaunchKernelGGL(interp_kernel_grouped<1>, grid, dim3(256), 0, st, djobs, dtab);
  else if (kmax <= 128)
    hipLaunchKernelGGL(interp_kernel_grouped<2>, grid, dim3(256), 0, st, djobs, dtab);
  else if (kmax <= 192)
    hipLaunchKernelGGL(interp_kernel_grouped<3>, grid, dim3(256), 0, st, djobs, dtab);
  else
    hipLaunchKernelGGL(interp_kernel_grouped<4>, grid, dim3(256), 0, st, djobs, dtab);
  ps.stop();
  return hipGetLastError();
}
