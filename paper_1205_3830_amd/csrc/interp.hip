// interp.hip -- the interpolation matrix of Sec. 2: solve R2 = R1 T by back
// substitution, each column on its own (the column-parallel "factorization
// of R" of Sec. 3.2), and write P = [I T] in the original column order.
//
// k <= 256: one wave per column of P.  The k right-hand-side entries of
// column j sit in the lanes (RR per lane, k <= 64 RR); step t divides entry t by the
// diagonal R1(t, t), broadcasts the quotient and updates the entries above
// it with column t of R1 (= column J[t] of R, a coalesced read that all
// columns share through the L2).  The read for step t-1 is issued before
// the arithmetic of step t.  Larger k (up to 1024), where k dependent steps
// per column would leave the device latency-bound: R1^-1 once (k columns),
// then P = R1^-1 R(0:k, :) as one GEMM on the FP64 matrix cores.
#include "rid_internal.hpp"

namespace {

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

template <int RR>
RID_DEV void interp_body(int64_t n, int64_t k, const double2 *__restrict__ R, int64_t ldr,
                         const int64_t *__restrict__ J, double2 *__restrict__ P, int64_t ldp,
                         const int *__restrict__ mark, int64_t bx) {
  __shared__ int64_t Js[64 * RR];
  for (int t = threadIdx.x; t < 64 * RR; t += blockDim.x) {
    int64_t jt = (t < k) ? J[t] : 0;
    if (jt < 0 || jt >= n) jt = 0;  // keeps every read inside R; such a P is meaningless
    Js[t] = jt;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t j = bx * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  double2 *pc = P + j * ldp;
  const int t0 = mark[j];
  if (t0 >= 0) {
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t s = lane + 64 * h;
      if (s < k) pc[s] = make_double2(s == t0 ? 1.0 : 0.0, 0.0);
    }
    return;
  }
  double2 r[RR];
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const int64_t s = lane + 64 * h;
    r[h] = (s < k) ? R[s + j * ldr] : make_double2(0.0, 0.0);
  }
  // column of R1 for the current step, prefetched one step ahead
  double2 rc[RR];
  {
    const double2 *cj = R + Js[k - 1] * ldr;
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t s = lane + 64 * h;
      rc[h] = (s < k) ? cj[s] : make_double2(0.0, 0.0);
    }
  }
  for (int64_t t = k - 1; t >= 0; --t) {
    double2 nx[RR];
    if (t > 0) {
      const double2 *cj = R + Js[t - 1] * ldr;
#pragma unroll
      for (int h = 0; h < RR; ++h) {
        const int64_t s = lane + 64 * h;
        nx[h] = (s < t) ? cj[s] : make_double2(0.0, 0.0);
      }
    }
    const int ht = static_cast<int>(t >> 6);
    const int lt = static_cast<int>(t & 63);
    double2 own = r[0];
    double2 dg = rc[0];
#pragma unroll
    for (int h = 1; h < RR; ++h)
      if (h == ht) {
        own = r[h];
        dg = rc[h];
      }
    const double ox = __shfl(own.x, lt, 64), oy = __shfl(own.y, lt, 64);
    const double dx = __shfl(dg.x, lt, 64), dy = __shfl(dg.y, lt, 64);
    const double den = dx * dx + dy * dy;
    const double tx = (ox * dx + oy * dy) / den;
    const double ty = (oy * dx - ox * dy) / den;
#pragma unroll
    for (int h = 0; h < RR; ++h) {
      const int64_t s = lane + 64 * h;
      if (s == t) {
        r[h] = make_double2(tx, ty);
      } else if (s < t) {
        r[h].x -= rc[h].x * tx - rc[h].y * ty;
        r[h].y -= rc[h].x * ty + rc[h].y * tx;
      }
    }
    if (t > 0) {
#pragma unroll
      for (int h = 0; h < RR; ++h) rc[h] = nx[h];
    }
  }
#pragma unroll
  for (int h = 0; h < RR; ++h) {
    const int64_t s = lane + 64 * h;
    if (s < k) pc[s] = r[h];
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

// A batch: block b solves the columns of quad tab[b].y of job tab[b].x.
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
    const double ox = __shfl(own.x, lt, 64), oy = __shfl(own.y, lt, 64);
    const double dx = __shfl(dg.x, lt, 64), dy = __shfl(dg.y, lt, 64);
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
  const unsigned nb = static_cast<unsigned>((n + 3) / 4);
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
