// sketch_srft.hip -- the randomization step with the paper's own operator,
// Y = S F D A (eqs. (4)-(7)), through a four-step split of the DFT instead
// of the explicit l x m operator.  With m = 8 m2 and row p = p2 + m2 p1,
//   Y(i, j) = sum_p e^{-2 pi i s_i p / m} d_p A(p, j)
//           = sum_{p2} e^{-2 pi i s_i p2 / m} Z_{t_i}(p2, j),
//   Z_t(p2, j) = sum_{p1 < 8} e^{-2 pi i t p1 / 8} d_{p2 + m2 p1} A(p2 + m2 p1, j),
// with t_i = s_i mod 8, because e^{-2 pi i s m2 p1 / m} = e^{-2 pi i s p1 / 8}.
// The 8-point DFTs (pass 1) read A once and write Z; the outer sums are one
// GEMM per residue t, K = m2, on the FP64 matrix cores (the sketch kernel
// with the twiddles T_t(r, p2) = e^{-2 pi i s p2 / m} of the rows r of group
// t as its operator), all eight in one launch.  That is 8 l m2 + O(m) complex multiply-adds per
// column instead of l m.  The draws are those of the explicit operator:
// d_p = e^{2 pi i phi_p}, phi_p the first uniform of Philox counter
// (p, 0, 0, 5), s_i = floor(u m) for the first uniform u of (i, 0, 0, 6).
#include <cmath>
#include <cstdlib>

#include "rid_internal.hpp"

namespace {

constexpr int R1 = 8;                         // the short DFT length
constexpr size_t Z_BLOCK_BYTES = size_t(1) << 31;  // column block of Z (pass 1 output)

// ---------------------------------------------------------------- host side
// The row draws s_i, for the host's launch sizes (the same Philox4x32-10
// block and uniform as the device's, in plain integer arithmetic).
void host_philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t n0 = uint32_t(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = uint32_t(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = uint32_t(p1);
    c[2] = n2;
    c[3] = uint32_t(p0);
  }
}

int64_t host_srft_row(uint64_t seed, int64_t i, int64_t m) {
  uint32_t c[4] = {uint32_t(uint64_t(i)), uint32_t(uint64_t(i) >> 32), 0u, 6u};
  host_philox10(c, uint32_t(seed), uint32_t(seed >> 32));
  const uint64_t x = ((uint64_t(c[1]) << 32) | c[0]) >> 12;
  const double u = double(2 * x + 1) * 0x1p-53;
  int64_t s = int64_t(std::floor(u * double(m)));
  return s >= m ? m - 1 : s;
}

struct Groups {
  int64_t off[R1 + 1];  // rows of residue t are off[t] .. off[t+1]-1 of the grouped order
};

Groups host_groups(uint64_t seed, int64_t l, int64_t m) {
  Groups g{};
  int64_t cnt[R1] = {0};
  for (int64_t i = 0; i < l; ++i) ++cnt[host_srft_row(seed, i, m) % R1];
  g.off[0] = 0;
  for (int t = 0; t < R1; ++t) g.off[t + 1] = g.off[t] + cnt[t];
  return g;
}

// ---------------------------------------------------------------- device side
// One workgroup: s_i for every row, then the rows grouped by t = s_i mod 8
// in increasing i (one thread per t scans the drawn rows): perm_i[r] is the
// original row and perm_s[r] its frequency, r in the grouped order.
__global__ __launch_bounds__(256) void srft_group_kernel(int64_t l, int64_t m, uint64_t seed,
                                                         Groups g, int64_t *__restrict__ perm_i,
                                                         int64_t *__restrict__ perm_s) {
  __shared__ int64_t s_sh[2048];
  for (int64_t i = threadIdx.x; i < l; i += blockDim.x) {
    int64_t s = static_cast<int64_t>(floor(rid_u1(seed, 6u, static_cast<uint64_t>(i)) *
                                           static_cast<double>(m)));
    s_sh[i] = s >= m ? m - 1 : s;
  }
  __syncthreads();
  if (threadIdx.x < R1) {
    const int t = threadIdx.x;
    int64_t o = g.off[t];
    for (int64_t i = 0; i < l; ++i) {
      if (s_sh[i] % R1 != t) continue;
      if (o < g.off[t + 1]) {  // the host's count bounds every write
        perm_i[o] = i;
        perm_s[o] = s_sh[i];
      }
      ++o;
    }
  }
}

// d_p = e^{2 pi i phi_p}, p < m.
__global__ __launch_bounds__(256) void srft_phase_kernel(int64_t m, uint64_t seed,
                                                         double2 *__restrict__ d) {
  for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < m;
       p += int64_t(gridDim.x) * blockDim.x) {
    const double ang =
        6.283185307179586476925286766559 * rid_u1(seed, 5u, static_cast<uint64_t>(p));
    d[p] = make_double2(cos(ang), sin(ang));
  }
}

// T(r, p2) = e^{-2 pi i (s_r p2 mod m) / m}, row-major l x m2.
__global__ __launch_bounds__(256) void srft_twiddle_kernel(int64_t l, int64_t m, int64_t m2,
                                                           const int64_t *__restrict__ perm_s,
                                                           double2 *__restrict__ T) {
  const int64_t total = l * m2;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / m2, p2 = e - r * m2;
    const uint64_t rr = (static_cast<uint64_t>(perm_s[r]) * static_cast<uint64_t>(p2)) %
                        static_cast<uint64_t>(m);
    const double ang = -6.283185307179586476925286766559 *
                       (static_cast<double>(rr) / static_cast<double>(m));
    T[e] = make_double2(cos(ang), sin(ang));
  }
}

RID_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
RID_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
RID_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
RID_DEV double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }  // -i a

// Pass 1 on columns j0 .. j0+nb-1: thread p2 of column j reads the eight
// rows p2 + m2 p1, multiplies them by d and writes their 8-point DFT
// (e^{-2 pi i t p1 / 8}) to Z_t(p2, j - j0), Z_t column-major m2 x nb.
template <class TA>
__global__ __launch_bounds__(256) void srft_dft8_kernel(int64_t m2, int64_t nb, int64_t j0,
                                                        const TA *__restrict__ A, int64_t lda,
                                                        const double2 *__restrict__ d,
                                                        double2 *__restrict__ Z) {
  const int64_t p2 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t jb = blockIdx.y;
  if (p2 >= m2) return;
  const TA *col = A + (j0 + jb) * lda;
  double2 v[R1];
#pragma unroll
  for (int p1 = 0; p1 < R1; ++p1) {
    const int64_t p = p2 + m2 * p1;
    v[p1] = cmul(ld_stream(col + p), d[p]);
  }
  // radix-2 decimation in time: E = DFT4(v0, v2, v4, v6), O = DFT4(v1, v3, v5, v7)
  auto dft4 = [](double2 a0, double2 a1, double2 a2, double2 a3, double2 *y) {
    const double2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3), b3 = csub(a1, a3);
    y[0] = cadd(b0, b2);
    y[2] = csub(b0, b2);
    y[1] = cadd(b1, mul_mi(b3));
    y[3] = csub(b1, mul_mi(b3));
  };
  double2 E[4], O[4];
  dft4(v[0], v[2], v[4], v[6], E);
  dft4(v[1], v[3], v[5], v[7], O);
  const double h = 0.70710678118654752440084436210485;  // cos(pi / 4)
  const double2 w[4] = {make_double2(1.0, 0.0), make_double2(h, -h), make_double2(0.0, -1.0),
                        make_double2(-h, -h)};  // e^{-2 pi i t / 8}
  double2 *z = Z + jb * m2 + p2;
  const int64_t plane = m2 * nb;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double2 o = cmul(w[t], O[t]);
    z[t * plane] = cadd(E[t], o);
    z[(t + 4) * plane] = csub(E[t], o);
  }
}

// ---------------------------------------------------------------- fused form
// When every residue group has at most 32 rows, the two passes fuse into one
// pass over A.  The grouped order is padded: group t owns rows t CAP ..
// t CAP + CAP - 1 (CAP = 8 TPG), its drawn rows first (increasing i), then
// padding (perm -1, zero twiddle row), so that each 8-row MFMA tile belongs
// to one group and takes its operand from that group's DFT output.
constexpr int FUSED_TPG_MAX = 4;

// RID_SRFT_TWO_PASS=1 in the environment selects the two-pass form even
// where the fused one applies (read at each call; the tests compare both).
bool srft_two_pass_forced() {
  const char *v = std::getenv("RID_SRFT_TWO_PASS");
  return v && v[0] == '1';
}

__global__ __launch_bounds__(256) void srft_group_pad_kernel(int64_t l, int64_t m, uint64_t seed,
                                                             int64_t cap, Groups g,
                                                             int64_t *__restrict__ perm_pad,
                                                             int64_t *__restrict__ s_pad) {
  __shared__ int64_t s_sh[2048];
  for (int64_t i = threadIdx.x; i < l; i += blockDim.x) {
    int64_t s = static_cast<int64_t>(floor(rid_u1(seed, 6u, static_cast<uint64_t>(i)) *
                                           static_cast<double>(m)));
    s_sh[i] = s >= m ? m - 1 : s;
  }
  for (int64_t r = threadIdx.x; r < R1 * cap; r += blockDim.x) {
    perm_pad[r] = -1;
    s_pad[r] = -1;
  }
  __syncthreads();
  if (threadIdx.x < R1) {
    const int t = threadIdx.x;
    int64_t o = 0;
    for (int64_t i = 0; i < l; ++i) {
      if (s_sh[i] % R1 != t) continue;
      if (o < cap && o < g.off[t + 1] - g.off[t]) {  // the host's counts bound every write
        perm_pad[t * cap + o] = i;
        s_pad[t * cap + o] = s_sh[i];
      }
      ++o;
    }
  }
}

// Tp(r, p2) = e^{-2 pi i (s_r p2 mod m) / m}, or 0 for a padding row; NR x m2.
__global__ __launch_bounds__(256) void srft_twiddle_pad_kernel(int64_t nr, int64_t m, int64_t m2,
                                                               const int64_t *__restrict__ s_pad,
                                                               double2 *__restrict__ Tp) {
  const int64_t total = nr * m2;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / m2, p2 = e - r * m2;
    const int64_t s = s_pad[r];
    if (s < 0) {
      Tp[e] = make_double2(0.0, 0.0);
      continue;
    }
    const uint64_t rr =
        (static_cast<uint64_t>(s) * static_cast<uint64_t>(p2)) % static_cast<uint64_t>(m);
    const double ang = -6.283185307179586476925286766559 *
                       (static_cast<double>(rr) / static_cast<double>(m));
    Tp[e] = make_double2(cos(ang), sin(ang));
  }
}

// In-place 8-point DFT, X_t = sum_p1 e^{-2 pi i t p1 / 8} v_p1 (radix 2, decimation in
// time: DFT4 of the even and of the odd samples).
RID_DEV void dft8(double2 (&v)[R1]) {
  auto dft4 = [](double2 a0, double2 a1, double2 a2, double2 a3, double2 *y) {
    const double2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3), b3 = csub(a1, a3);
    y[0] = cadd(b0, b2);
    y[2] = csub(b0, b2);
    y[1] = cadd(b1, mul_mi(b3));
    y[3] = csub(b1, mul_mi(b3));
  };
  double2 E[4], O[4];
  dft4(v[0], v[2], v[4], v[6], E);
  dft4(v[1], v[3], v[5], v[7], O);
  const double h = 0.70710678118654752440084436210485;  // cos(pi / 4)
  const double2 w[4] = {make_double2(1.0, 0.0), make_double2(h, -h), make_double2(0.0, -1.0),
                        make_double2(-h, -h)};  // e^{-2 pi i t / 8}
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double2 o = cmul(w[t], O[t]);
    v[t] = cadd(E[t], o);
    v[t + 4] = csub(E[t], o);
  }
}

typedef double fd4 __attribute__((ext_vector_type(4)));

// The fused sketch on the FP64 matrix cores (v_mfma_f64_16x16x4f64), in the
// real embedding of the complex product like the Gaussian sketch: a workgroup
// of 4 waves owns 64 columns and a K range of p2; each wave owns 16 columns.
// A K step covers 8 values of p2.  Lane (r16 = lane % 16, q = lane / 16)
// reads, for its column r16 and its two rows p2 = p0 + 2q + u (u = 0, 1),
// the eight rows p2 + m2 p1 of A, multiplies them by d (staged in LDS) and
// takes their 8-point DFTs: the values Z_t(p2, col) for every residue t.
// MFMA (u, re/im) then uses k-slot q for real K row 2 (p0 + 2q + u) + re/im,
// so tile tau = t TPG + jj (complex rows 8 tau .. 8 tau + 7 of the padded
// order, all in group t) takes its B operand straight from Z_t, and its A
// operand from the twiddle slab (staged in LDS, double buffered, row stride
// 9).  The next step's A rows, twiddles and d are loaded during the current
// step.  Partials: part[split][column][real row], ld 2 NR.
template <int TPG, class TA>
__global__ __launch_bounds__(256) void srft_fused_kernel(int64_t m2, int64_t n,
                                                         const TA *__restrict__ A, int64_t lda,
                                                         const double2 *__restrict__ d,
                                                         const double2 *__restrict__ Tp,
                                                         double *__restrict__ part,
                                                         int64_t pchunk) {
  constexpr int NT = R1 * TPG;                // MFMA tiles (8 complex rows each)
  constexpr int NR = 8 * NT;                  // complex rows of Tp
  constexpr int KS = 8;                       // p2 values per K step
  constexpr int RS = KS + 1;                  // LDS row stride of the twiddle slab
  constexpr int PER = (NR * KS + 255) / 256;  // twiddle entries staged per thread
  __shared__ double2 gs[2][NR * RS];
  __shared__ double2 ds[2][KS * R1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int r16 = lane & 15;
  const int c = lane & 1;
  const int64_t jcol = blockIdx.x * int64_t(64) + wave * 16 + r16;
  const bool colok = jcol < n;
  const int64_t pbeg = blockIdx.y * pchunk;
  const int64_t pend = min(m2, pbeg + pchunk);

  fd4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = fd4{0.0, 0.0, 0.0, 0.0};

  const TA *Acol = A + (colok ? jcol : 0) * lda;
  double2 stg[PER];
  double2 dstg = make_double2(0.0, 0.0);
  auto load_g = [&](int64_t p0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      const int row = e / KS, col = e % KS;
      const int64_t p = p0 + col;
      stg[r] = (e < NR * KS && p < pend) ? Tp[row * m2 + p] : make_double2(0.0, 0.0);
    }
    if (tid < KS * R1) {
      const int64_t p = p0 + tid % KS;
      dstg = p < pend ? d[p + m2 * (tid / KS)] : make_double2(0.0, 0.0);
    }
  };
  auto store_g = [&](int b) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      if (e < NR * KS) gs[b][(e / KS) * RS + e % KS] = stg[r];
    }
    if (tid < KS * R1) ds[b][tid] = dstg;
  };
  auto load_a = [&](int64_t p0, double2 (&v)[2][R1]) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t p2 = p0 + 2 * q + u;
      const bool ok = colok && p2 < pend;
#pragma unroll
      for (int p1 = 0; p1 < R1; ++p1)
        v[u][p1] = ok ? ld_stream(Acol + p2 + m2 * p1) : make_double2(0.0, 0.0);
    }
  };

  double2 va[2][R1], vn[2][R1];
  load_g(pbeg);
  store_g(0);
  load_a(pbeg, va);
  // Wait for the first step's loads here: loads still pending into va when
  // the loop starts would make every iteration wait for all outstanding
  // loads -- the next step's prefetch included -- before its first use of va.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int b = 0;
  for (int64_t p0 = pbeg; p0 < pend; p0 += KS) {
    const bool more = p0 + KS < pend;
    if (more) {
      load_g(p0 + KS);
      load_a(p0 + KS, vn);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int p1 = 0; p1 < R1; ++p1) va[u][p1] = cmul(va[u][p1], ds[b][p1 * KS + 2 * q + u]);
      dft8(va[u]);  // va[u][t] = Z_t(p0 + 2q + u, column)
    }
    // for each (u, jj): the real-part products of the eight groups' tiles,
    // then their imaginary-part products, so that consecutive MFMAs write
    // different accumulators (one wave per SIMD leaves no other wave to
    // cover a dependent MFMA's latency)
    const double2 *gb = gs[b];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int jj = 0; jj < TPG; ++jj) {
        double o0[R1], o1[R1];
#pragma unroll
        for (int t = 0; t < R1; ++t) {
          const int row = 8 * (t * TPG + jj) + (r16 >> 1);
          const double2 g = gb[row * RS + 2 * q + u];
          // row 2i (c = 0): [Re g, -Im g];  row 2i+1 (c = 1): [Im g, Re g]
          o0[t] = c ? g.y : g.x;
          o1[t] = c ? g.x : -g.y;
        }
#pragma unroll
        for (int t = 0; t < R1; ++t)
          acc[t * TPG + jj] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(o0[t], va[u][t].x, acc[t * TPG + jj], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);  // keep the two sweeps apart
#pragma unroll
        for (int t = 0; t < R1; ++t)
          acc[t * TPG + jj] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(o1[t], va[u][t].y, acc[t * TPG + jj], 0, 0, 0);
      }
    }
    if (more) {
      store_g(b ^ 1);
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int p1 = 0; p1 < R1; ++p1) va[u][p1] = vn[u][p1];
    }
    __syncthreads();
    b ^= 1;
  }
  if (!colok) return;
  // D layout of the f64 16x16x4 MFMA: lane, register r -> row 4r + lane/16,
  // column lane % 16.
  double *o = part + blockIdx.y * (2 * NR * n) + jcol * (2 * NR);
#pragma unroll
  for (int tau = 0; tau < NT; ++tau)
#pragma unroll
    for (int r = 0; r < 4; ++r) o[tau * 16 + 4 * r + q] = acc[tau][r];
}

// Y(perm_pad[r], j) = sum over the splits of the padded row r; padding rows
// are skipped.
__global__ __launch_bounds__(256) void srft_fused_reduce_kernel(
    int64_t nr, int64_t n, int64_t l, int S, const double *__restrict__ part,
    const int64_t *__restrict__ perm_pad, double2 *__restrict__ Y, int64_t ldy) {
  const int64_t total = nr * n;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = e / nr, r = e - j * nr;
    const int64_t i = perm_pad[r];
    if (i < 0 || i >= l) continue;
    const double *pt = part + j * 2 * nr + 2 * r;
    double re = 0.0, im = 0.0;
    for (int sp = 0; sp < S; ++sp) {
      re += pt[sp * 2 * nr * n];
      im += pt[sp * 2 * nr * n + 1];
    }
    Y[j * ldy + i] = make_double2(re, im);
  }
}

struct FusedPlan {
  int64_t nbx, S, pchunk;
};

FusedPlan plan_fused(int64_t m2, int64_t n) {
  FusedPlan p;
  p.nbx = (n + 63) / 64;
  int64_t S = (1024 + p.nbx - 1) / p.nbx;
  const int64_t maxS = (m2 + 127) / 128;  // at least 16 K steps per split
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  int64_t pchunk = (m2 + S - 1) / S;
  pchunk = (pchunk + 7) / 8 * 8;
  if ((m2 + pchunk - 1) / pchunk > 65535) pchunk = ((m2 + 65534) / 65535 + 7) / 8 * 8;
  p.S = (m2 + pchunk - 1) / pchunk;
  p.pchunk = pchunk;
  return p;
}

struct SrftWs {
  int64_t *perm_i, *perm_s;
  double2 *d, *T, *Z;
  void *part;
  int64_t nb;  // columns per block of Z
  // fused form: padded grouped order, its twiddles and split partials
  int64_t *perm_pad, *s_pad;
  double2 *Tp;
  double *fpart;
};

int64_t block_cols(int64_t m, int64_t n) {
  int64_t nb = static_cast<int64_t>(Z_BLOCK_BYTES / (size_t(m) * sizeof(double2)));
  if (nb < 1) nb = 1;
  if (nb > n) nb = n;
  if (nb > 65535) nb = 65535;  // grid y of pass 1
  return nb;
}

template <class C>
SrftWs carve_srft(C &c, int64_t m, int64_t n, int64_t l) {
  SrftWs w;
  const int64_t m2 = m / R1;
  w.nb = block_cols(m, n);
  w.perm_i = c.template take<int64_t>(size_t(l));
  w.perm_s = c.template take<int64_t>(size_t(l));
  w.d = c.template take<double2>(size_t(m));
  w.T = c.template take<double2>(size_t(l) * size_t(m2));
  w.Z = c.template take<double2>(size_t(m) * size_t(w.nb));
  w.part = c.template take<char>(srft_gemm_ws_bytes(m2, w.nb, l));
  const int64_t nrmax = 8 * R1 * FUSED_TPG_MAX;
  w.perm_pad = c.template take<int64_t>(size_t(nrmax));
  w.s_pad = c.template take<int64_t>(size_t(nrmax));
  w.Tp = c.template take<double2>(size_t(nrmax) * size_t(m2));
  w.fpart = c.template take<double>(size_t(plan_fused(m2, n).S) * 2 * size_t(nrmax) * size_t(n));
  return w;
}

unsigned grid_1d(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

bool srft_fft_ok(rid_prec prec, int64_t m, int64_t l) {
  return prec == RID_FP64 && m >= R1 && m % R1 == 0 && m <= 0x7FFFFFFFll && l <= 2048;
}

size_t srft_sketch_ws_bytes(int64_t m, int64_t n, int64_t l) {
  WsCarve c(nullptr);
  carve_srft(c, m, n, l);
  return c.off + 256;
}

hipError_t launch_srft_sketch(hipStream_t st, rid_dtype dtype, int64_t m, int64_t n, int64_t l,
                              const void *A, int64_t lda, uint64_t seed, double2 *Y, int64_t ldy,
                              void *ws, RidProf *prof) {
  if (n == 0 || l == 0) return hipSuccess;
  const int64_t m2 = m / R1;
  WsCarve c(ws);
  const SrftWs w = carve_srft(c, m, n, l);
  // every row's group; the host's copy of the draws sizes the launches
  const Groups g = host_groups(seed, l, m);
  int64_t lmax = 0;
  for (int t = 0; t < R1; ++t) lmax = std::max(lmax, g.off[t + 1] - g.off[t]);
  const int tpg = static_cast<int>((lmax + 7) / 8);
  if (tpg <= FUSED_TPG_MAX && !srft_two_pass_forced()) {
    const int64_t cap = 8 * tpg, nr = R1 * cap;
    hipLaunchKernelGGL(srft_group_pad_kernel, dim3(1), dim3(256), 0, st, l, m, seed, cap, g,
                       w.perm_pad, w.s_pad);
    hipLaunchKernelGGL(srft_phase_kernel, dim3(grid_1d(m)), dim3(256), 0, st, m, seed, w.d);
    hipLaunchKernelGGL(srft_twiddle_pad_kernel, dim3(grid_1d(nr * m2)), dim3(256), 0, st, nr, m,
                       m2, w.s_pad, w.Tp);
    const FusedPlan fp = plan_fused(m2, n);
    const dim3 grid(static_cast<unsigned>(fp.nbx), static_cast<unsigned>(fp.S));
    {
      ProfScope ps(prof, st, RID_KERNEL_SKETCH);
#define RID_FUSED(T)                                                                         \
  case T:                                                                                    \
    if (dtype == RID_C64)                                                                    \
      hipLaunchKernelGGL((srft_fused_kernel<T, float2>), grid, dim3(256), 0, st, m2, n,      \
                         static_cast<const float2 *>(A), lda, w.d, w.Tp, w.fpart, fp.pchunk); \
    else                                                                                     \
      hipLaunchKernelGGL((srft_fused_kernel<T, double2>), grid, dim3(256), 0, st, m2, n,     \
                         static_cast<const double2 *>(A), lda, w.d, w.Tp, w.fpart,           \
                         fp.pchunk);                                                         \
    break;
      switch (tpg) {
        RID_FUSED(1) RID_FUSED(2) RID_FUSED(3) RID_FUSED(4)
        default:
          return hipErrorInvalidValue;
      }
#undef RID_FUSED
      ps.stop();
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(srft_fused_reduce_kernel, dim3(grid_1d(nr * n)), dim3(256), 0, st, nr, n,
                       l, static_cast<int>(fp.S), w.fpart, w.perm_pad, Y, ldy);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(srft_group_kernel, dim3(1), dim3(256), 0, st, l, m, seed, g, w.perm_i,
                     w.perm_s);
  hipLaunchKernelGGL(srft_phase_kernel, dim3(grid_1d(m)), dim3(256), 0, st, m, seed, w.d);
  hipLaunchKernelGGL(srft_twiddle_kernel, dim3(grid_1d(l * m2)), dim3(256), 0, st, l, m, m2,
                     w.perm_s, w.T);
  hipError_t e = hipGetLastError();
  for (int64_t j0 = 0; j0 < n && e == hipSuccess; j0 += w.nb) {
    const int64_t nb = std::min(w.nb, n - j0);
    const dim3 grid(static_cast<unsigned>((m2 + 255) / 256), static_cast<unsigned>(nb));
    if (dtype == RID_C64)
      hipLaunchKernelGGL(srft_dft8_kernel<float2>, grid, dim3(256), 0, st, m2, nb, j0,
                         static_cast<const float2 *>(A), lda, w.d, w.Z);
    else
      hipLaunchKernelGGL(srft_dft8_kernel<double2>, grid, dim3(256), 0, st, m2, nb, j0,
                         static_cast<const double2 *>(A), lda, w.d, w.Z);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = launch_srft_gemm(st, m2, nb, j0, g.off, w.Z, w.T, w.perm_i, Y, ldy, w.part, prof);
  }
  return e;
}
