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

struct SrftWs {
  int64_t *perm_i, *perm_s;
  double2 *d, *T, *Z;
  void *part;
  int64_t nb;  // columns per block of Z
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
