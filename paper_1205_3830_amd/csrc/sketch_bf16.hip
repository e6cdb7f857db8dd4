// sketch_bf16.hip -- randomization step Y = G A (Sec. 2) with products on the
// bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16), each operand split into
// NT bfloat16 terms (round to nearest at each step), accumulated in FP32
// within a K split; the K splits are summed in double into the complex128 Y.
//   NT = 3: x = x_h + x_m + x_l (24 significant bits), the six leading cross
//           products a_h b_h + a_h b_m + a_m b_h + a_h b_l + a_m b_m + a_l b_h;
//           the dropped ones are below 2^-24 relative: FP32-level error.
//   NT = 2: x = x_h + x_l (16 significant bits), the three products
//           a_h b_h + a_h b_l + a_l b_h; the dropped a_l b_l is below 2^-16
//           relative: error near 2^-16, at half the matrix-core work.
// The pivoted QR, the solve and the residual that follow stay in double.
//
// Real embedding as in the other sketches, on the A side: [Yr Yi] (l x 2n) =
// [Gr Gi] (l x 2m) Ae (2m x 2n), with the 2 x 2 blocks [[Re a, Im a],
// [-Im a, Re a]] of Ae built per lane from the A entries it loaded, once per
// K step.  Operand layouts of the bf16 16x16x32 MFMA (measured on gfx950):
// lane l supplies row l % 16 of the A operand (and column l % 16 of the B
// operand) at k = 8 (l / 16) .. 8 (l / 16) + 7; D lane l, register r is row
// 4 (l / 16) + r, column l % 16.  So one MFMA covers 16 complex rows of A: a
// lane's four consecutive complex entries of its column give its eight
// k-slots (k-index 2p + e), and row i of [Gr Gi] over those k-slots is 16
// contiguous bytes of a pre-split plane; real column r16 of a tile is part
// r16 & 1 of complex column r16 >> 1.
//
// G is split once per call into NT bf16 planes of [Gr Gi] (row-major,
// 2 m_pad columns, zero padding), reused by every column block.  A
// workgroup (8 waves) owns 128 columns of A -- 2 groups of 8 per wave, so
// each G operand read from LDS feeds two MFMA sets -- and RT 16-row tiles of
// Y.  Per K step of 16 complex rows the workgroup stages the NT planes'
// slab in LDS (double buffered, one barrier per step; the next slab and the
// next A entries are loaded into registers while the current step computes).  The
// staged slab is l rows, half of the 2l rows a G-side embedding stages for
// the same 128 columns, so the slab reads from L2 and the last-level cache
// per matrix-core operation are halved.
#include "rid_internal.hpp"

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BF_RT_MAX = 14;  // row tiles of Y per workgroup (LDS: 3 KB per tile)

// The NT leading bf16 terms of v: t[0] = bf16(v), t[s] = bf16 of what the
// earlier terms leave (each residual formed exactly in double).
template <int NT>
RID_DEV void split_terms(double v, __bf16 (&t)[NT]) {
  double r = v;
#pragma unroll
  for (int s = 0; s < NT; ++s) {
    t[s] = static_cast<__bf16>(static_cast<float>(r));
    r -= static_cast<double>(static_cast<float>(t[s]));
  }
}

// Gs plane s (s < NT, at s * pstride), entry (i, kappa) at i * ldk + kappa:
// bf16 term s of [Gr Gi](i, kappa) -- Re G(i, kappa/2) for even,
// Im G(i, kappa/2) for odd kappa -- for i < rows_pad, kappa < ldk (zero
// outside l x 2m).  One thread per complex entry (i, p).
// Entries first, first + stride, ... of the rows_pad x mpad grid.
template <int NT>
RID_DEV void split_planes(int64_t l, int64_t m, int64_t rows_pad, int64_t mpad,
                          const double2 *__restrict__ G, int64_t ldg, __bf16 *__restrict__ Gs,
                          int64_t ldk, int64_t pstride, int64_t first, int64_t stride) {
  const int64_t total = rows_pad * mpad;
  for (int64_t e = first; e < total; e += stride) {
    const int64_t i = e / mpad;
    const int64_t p = e - i * mpad;
    const double2 g = (i < l && p < m) ? G[i * ldg + p] : make_double2(0.0, 0.0);
    const double v[2] = {g.x, g.y};
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      __bf16 t[NT];
      split_terms<NT>(v[part], t);
      const int64_t at = i * ldk + 2 * p + part;
#pragma unroll
      for (int s = 0; s < NT; ++s) Gs[s * pstride + at] = t[s];
    }
  }
}

template <int NT>
__global__ __launch_bounds__(256) void bf16_split_kernel(int64_t l, int64_t m, int64_t rows_pad,
                                                         int64_t mpad,
                                                         const double2 *__restrict__ G,
                                                         int64_t ldg, __bf16 *__restrict__ Gs,
                                                         int64_t ldk, int64_t pstride) {
  split_planes<NT>(l, m, rows_pad, mpad, G, ldg, Gs, ldk, pstride,
                   blockIdx.x * int64_t(blockDim.x) + threadIdx.x,
                   int64_t(gridDim.x) * blockDim.x);
}

// A batch: workgroup b takes entry (job, block, blocks-of-job) of tab.
template <int NT>
__global__ __launch_bounds__(256) void bf16_split_grouped(const SketchJob *__restrict__ jobs,
                                                          const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const SketchJob &j = jobs[e.x];
  split_planes<NT>(j.l, j.m, j.prow, j.ldk / 2, j.G, j.ldg, static_cast<__bf16 *>(j.planes),
                   j.ldk, j.pstride, int64_t(e.y) * 256 + threadIdx.x, int64_t(e.z) * 256);
}

// The lane's four entries of A in their stored type (converted later, by
// to_floats: converting right after the load would make the wave wait for
// the load there, serialising the prefetch with the step's products).
// WHOLE: a lane whose four entries are all in range loads them without
// per-entry guards (wide loads, no branch per entry).  Measured at 131072 x
// 16384, l = 108: the two-term sketch 7.9 -> 6.4 ms with it, the three-term
// one 10.7 -> 12.3 ms, so only the two-term kernel takes it.
template <class TA, bool WHOLE>
RID_DEV void load_a(const TA *Acol, int64_t pb, int64_t pend, bool ok, TA (&v)[4]) {
  if (WHOLE && ok && pb + 4 <= pend) {
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = Acol[pb + u];
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (ok && pb + u < pend) ? Acol[pb + u] : zero_of<TA>();
  }
}

template <class TA>
RID_DEV void to_floats(const TA (&a)[4], float (&v)[8]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 d = to_d2(a[u]);
    v[2 * u] = static_cast<float>(d.x);
    v[2 * u + 1] = static_cast<float>(d.y);
  }
}

// The NT bf16 terms of eight floats (residuals exact in float).
template <int NT>
RID_DEV void split_vec(const float (&v)[8], bf8 (&t)[NT]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float r = v[e];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const __bf16 x = static_cast<__bf16>(r);
      t[s][e] = x;
      r -= static_cast<float>(x);
    }
  }
}

// Block (bx, by, bz): columns [128 bx, 128 bx + 128), K split by (rows
// [by pchunk, ...) of A), row tiles [RT bz, RT bz + RT) of Y.
template <int RT, class TA, int NT>
RID_DEV void sketch_bf16_body(int64_t m, int64_t n, int64_t l, const TA *__restrict__ A,
                              int64_t lda, const __bf16 *__restrict__ Gs, int64_t ldk,
                              int64_t pstride, float *__restrict__ out, int64_t ldo,
                              int64_t split_stride, int64_t pchunk, int64_t bx, int64_t by,
                              int64_t bz) {
  constexpr int NTH = 512;
  constexpr int ROWS = 16 * RT;                 // rows of Y (and of the planes) in the slab
  constexpr int CHUNKS = NT * ROWS * 4;         // 16-byte pieces of the slab (NT planes)
  constexpr int PER = (CHUNKS + NTH - 1) / NTH; // pieces staged per thread
  __shared__ uint4 gsl[2][NT][ROWS][4];         // [buffer][plane][row][k-group of 8]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int r16 = lane & 15;
  const int c = r16 & 1;
  const int64_t i0 = bz * ROWS;                 // first row of Y of the slab
  const int64_t pbeg = by * pchunk;
  const int64_t pend = min(m, pbeg + pchunk);
  int64_t jcol[2];
  bool ok[2];
  const TA *Acol[2];
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    jcol[g] = bx * 128 + wave * 16 + g * 8 + (r16 >> 1);
    ok[g] = jcol[g] < n;
    Acol[g] = A + (ok[g] ? jcol[g] : 0) * lda;
  }
  f4 acc[2][RT];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[g][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  const int64_t rows_all = ((l + ROWS - 1) / ROWS) * ROWS;  // rows of the planes
  uint4 stg[PER];
  auto load_slab = [&](int64_t p0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + NTH * r;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (e < CHUNKS && p0 < pend) {
        const int plane = e / (ROWS * 4);
        const int rem = e - plane * ROWS * 4;
        const int row = rem >> 2, kg = rem & 3;
        const int64_t i = i0 + row;
        if (i < rows_all) {
          const __bf16 *src = Gs + plane * pstride + i * ldk + 2 * p0 + 8 * kg;
          v = *reinterpret_cast<const uint4 *>(src);
        }
      }
      stg[r] = v;
    }
  };
  auto store_slab = [&](int b) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + NTH * r;
      if (e < CHUNKS) {
        const int plane = e / (ROWS * 4);
        const int rem = e - plane * ROWS * 4;
        gsl[b][plane][rem >> 2][rem & 3] = stg[r];
      }
    }
  };

  float av[2][8];
  TA an[2][4];
  load_slab(pbeg);
  store_slab(0);
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    load_a<TA, NT == 2>(Acol[g], pbeg + 4 * q, pend, ok[g], an[g]);
    to_floats(an[g], av[g]);
  }
  // nothing may be pending into av when the loop starts (it would make every
  // step wait for its own prefetch before the first product)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int b = 0;
  for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
    const bool more = p0 + 16 < pend;
    if (more) {
      load_slab(p0 + 16);
#pragma unroll
      for (int g = 0; g < 2; ++g) load_a<TA, NT == 2>(Acol[g], p0 + 16 + 4 * q, pend, ok[g], an[g]);
    }
    // B operand: k-index 2p (e = 0) carries [Re a, Im a] for parts c = 0, 1;
    // k-index 2p+1 carries [-Im a, Re a]; then its NT bf16 terms
    bf8 bt[2][NT];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      float bv[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bv[2 * u] = c ? av[g][2 * u + 1] : av[g][2 * u];
        bv[2 * u + 1] = c ? av[g][2 * u] : -av[g][2 * u + 1];
      }
      split_vec<NT>(bv, bt[g]);
    }
    // tiles in groups of TG: each product sweeps TG tiles x 2 column groups,
    // so consecutive MFMAs use 2 TG different accumulators (no back-to-back
    // dependence); smallest products first
    constexpr int TG = 4;
#pragma unroll
    for (int t0 = 0; t0 < RT; t0 += TG) {
      bf8 at[NT][TG];
#pragma unroll
      for (int u = 0; u < TG; ++u) {
        if (t0 + u < RT) {
#pragma unroll
          for (int s = 0; s < NT; ++s)
            at[s][u] = __builtin_bit_cast(bf8, gsl[b][s][16 * (t0 + u) + r16][q]);
        }
      }
      // products of G's term SA and A's term SB, orders summing to <= NT - 1
#define RID_BF_PRODUCT(SA, SB)                                                        \
  _Pragma("unroll") for (int u = 0; u < TG; ++u) {                                   \
    if (t0 + u < RT) {                                                               \
      _Pragma("unroll") for (int g = 0; g < 2; ++g) acc[g][t0 + u] =                 \
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(at[SA][u], bt[g][SB], acc[g][t0 + u], \
                                                  0, 0, 0);                          \
    }                                                                                \
  }
      if constexpr (NT == 3) {
        RID_BF_PRODUCT(2, 0)
        RID_BF_PRODUCT(1, 1)
        RID_BF_PRODUCT(0, 2)
        RID_BF_PRODUCT(1, 0)
        RID_BF_PRODUCT(0, 1)
        RID_BF_PRODUCT(0, 0)
      } else {
        RID_BF_PRODUCT(1, 0)
        RID_BF_PRODUCT(0, 1)
        RID_BF_PRODUCT(0, 0)
      }
#undef RID_BF_PRODUCT
    }
    if (more) {
      store_slab(b ^ 1);
#pragma unroll
      for (int g = 0; g < 2; ++g) to_floats(an[g], av[g]);
    }
    __syncthreads();  // the next slab is in place, and this one no longer read
    b ^= 1;
  }
  // `out` holds the real parts of Y's rows at even and the imaginary parts
  // at odd offsets of each column (ldo floats apart)
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    if (!ok[g]) continue;
    float *o = out + by * split_stride + jcol[g] * ldo;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + int64_t(t) * 16 + 4 * q + r;
        if (i < l) o[2 * i + c] = acc[g][t][r];
      }
  }
}

template <int RT, class TA, int NT>
__global__ __launch_bounds__(512) void sketch_bf16_kernel(
    int64_t m, int64_t n, int64_t l, const TA *__restrict__ A, int64_t lda,
    const __bf16 *__restrict__ Gs, int64_t ldk, int64_t pstride, float *__restrict__ out,
    int64_t ldo, int64_t split_stride, int64_t pchunk) {
  sketch_bf16_body<RT, TA, NT>(m, n, l, A, lda, Gs, ldk, pstride, out, ldo, split_stride,
                               pchunk, blockIdx.x, blockIdx.y, blockIdx.z);
}

// A batch: workgroup b takes entry (job, bx, split) of tab; the job's planes
// have 16 RT rows.
template <int RT, class TA, int NT>
__global__ __launch_bounds__(512) void sketch_bf16_kernel_grouped(
    const SketchJob *__restrict__ jobs, const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const SketchJob &j = jobs[e.x];
  sketch_bf16_body<RT, TA, NT>(j.m, j.n, j.l, static_cast<const TA *>(j.A), j.lda,
                               static_cast<const __bf16 *>(j.planes), j.ldk, j.pstride,
                               static_cast<float *>(j.part), 2 * j.l, 2 * j.l * j.n, j.pchunk,
                               e.y, e.z, 0);
}

// A batch: Y = the sum over the job's splits (in order, in double) of its
// partials; workgroup b takes entry (job, block, blocks-of-job) of tab.
__global__ __launch_bounds__(256) void bf16_reduce_grouped(const SketchJob *__restrict__ jobs,
                                                           const int4 *__restrict__ tab) {
  const int4 en = tab[blockIdx.x];
  const SketchJob &jb = jobs[en.x];
  const int64_t total = 2 * jb.l * jb.n;
  const float *part = static_cast<const float *>(jb.part);
  double *Y = reinterpret_cast<double *>(jb.Y);
  for (int64_t e = int64_t(en.y) * 256 + threadIdx.x; e < total; e += int64_t(en.z) * 256) {
    double s = 0.0;
    for (int64_t sp = 0; sp < jb.S; ++sp) s += static_cast<double>(part[sp * total + e]);
    Y[e] = s;
  }
}

// Y(mu, j) = sum over splits (in order, in double) of part[s](mu, j).
__global__ __launch_bounds__(256) void bf16_reduce_kernel(int64_t rows, int64_t n, int S,
                                                          const float *__restrict__ part,
                                                          double *__restrict__ Y, int64_t ldy2) {
  const int64_t total = rows * n;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = e / rows;
    const int64_t mu = e - j * rows;
    double s = 0.0;
    for (int sp = 0; sp < S; ++sp) s += static_cast<double>(part[sp * total + e]);
    Y[j * ldy2 + mu] = s;
  }
}

struct BfPlan {
  int RT;          // row tiles of Y per workgroup
  int nbz;         // workgroups along the rows of Y
  int64_t nbx;     // workgroups along the columns (128 each)
  int S;           // K splits
  int64_t pchunk;  // rows of A per split (multiple of 16)
  int64_t mpad;    // complex columns of the planes (multiple of 16)
  int64_t rows_pad;  // rows of the planes
  int64_t ldk, pstride;
};

BfPlan plan_bf16(int64_t m, int64_t n, int64_t l) {
  BfPlan p;
  const int64_t tiles = (l + 15) / 16;
  p.nbz = static_cast<int>((tiles + BF_RT_MAX - 1) / BF_RT_MAX);
  p.RT = static_cast<int>((tiles + p.nbz - 1) / p.nbz);
  p.nbx = (n + 127) / 128;
  const int64_t base = p.nbx * p.nbz;
  int64_t S = (2048 + base - 1) / base;
  const int64_t maxS = (m + 255) / 256;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  int64_t pchunk = (m + S - 1) / S;
  pchunk = (pchunk + 15) / 16 * 16;
  if (pchunk < 16) pchunk = 16;
  if (rid_tl_short_blocks && pchunk > RID_SPLIT_ROWS_MAX) pchunk = RID_SPLIT_ROWS_MAX;
  if ((m + pchunk - 1) / pchunk > 65535) pchunk = ((m + 65534) / 65535 + 15) / 16 * 16;
  p.S = static_cast<int>((m + pchunk - 1) / pchunk);
  if (p.S < 1) p.S = 1;
  p.pchunk = pchunk;
  p.mpad = ((m + 15) / 16) * 16;
  p.rows_pad = int64_t(p.nbz) * p.RT * 16;  // every slab row exists
  p.ldk = 2 * p.mpad;
  p.pstride = p.rows_pad * p.ldk;
  return p;
}

template <int RT, class TA, int NT>
void launch_bf16_rt(hipStream_t st, const BfPlan &p, int64_t m, int64_t n, int64_t l,
                    const TA *A, int64_t lda, const __bf16 *Gs, float *part) {
  dim3 grid(static_cast<unsigned>(p.nbx), static_cast<unsigned>(p.S),
            static_cast<unsigned>(p.nbz));
  hipLaunchKernelGGL((sketch_bf16_kernel<RT, TA, NT>), grid, dim3(512), 0, st, m, n, l, A, lda,
                     Gs, p.ldk, p.pstride, part, 2 * l, 2 * l * n, p.pchunk);
}

template <class TA, int NT>
hipError_t launch_bf16_terms(hipStream_t st, int64_t m, int64_t n, int64_t l, const TA *A,
                             int64_t lda, const double2 *G, int64_t ldg, double2 *Y,
                             int64_t ldy, void *ws, RidProf *prof) {
  if (n == 0 || l == 0) return hipSuccess;
  if (m == 0) return launch_zero(st, l, n, Y, ldy);
  const BfPlan p = plan_bf16(m, n, l);
  WsCarve c(ws);
  __bf16 *Gs = c.take<__bf16>(3 * size_t(p.pstride));
  float *part = c.take<float>(size_t(p.S) * size_t(2 * l) * size_t(n));
  {
    const int64_t total = p.rows_pad * p.mpad;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((bf16_split_kernel<NT>), dim3(static_cast<unsigned>(blocks)), dim3(256),
                       0, st, l, m, p.rows_pad, p.mpad, G, ldg, Gs, p.ldk, p.pstride);
  }
  ProfScope ps(prof, st, RID_KERNEL_SKETCH);
  switch (p.RT) {
#define RID_BF_CASE(X)                                               \
  case X:                                                            \
    launch_bf16_rt<X, TA, NT>(st, p, m, n, l, A, lda, Gs, part);     \
    break;
    RID_BF_CASE(1) RID_BF_CASE(2) RID_BF_CASE(3) RID_BF_CASE(4) RID_BF_CASE(5) RID_BF_CASE(6)
    RID_BF_CASE(7) RID_BF_CASE(8) RID_BF_CASE(9) RID_BF_CASE(10) RID_BF_CASE(11)
    RID_BF_CASE(12) RID_BF_CASE(13) RID_BF_CASE(14)
#undef RID_BF_CASE
    default:
      return hipErrorInvalidValue;
  }
  ps.stop();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = 2 * l * n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(bf16_reduce_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     2 * l, n, p.S, part, reinterpret_cast<double *>(Y), 2 * ldy);
  return hipGetLastError();
}

}  // namespace

size_t sketch_bf16_ws_bytes(int64_t m, int64_t n, int64_t l) {
  const BfPlan p = plan_bf16(m, n, l);
  WsCarve c(nullptr);
  c.take<__bf16>(3 * size_t(p.pstride));
  c.take<float>(size_t(p.S) * size_t(2 * l) * size_t(n));
  return c.off;
}

template <class TA>
hipError_t launch_sketch_bf16(hipStream_t st, int terms, int64_t m, int64_t n, int64_t l,
                              const TA *A, int64_t lda, const double2 *G, int64_t ldg,
                              double2 *Y, int64_t ldy, void *ws, RidProf *prof) {
  if (terms == 2)
    return launch_bf16_terms<TA, 2>(st, m, n, l, A, lda, G, ldg, Y, ldy, ws, prof);
  if (terms == 3)
    return launch_bf16_terms<TA, 3>(st, m, n, l, A, lda, G, ldg, Y, ldy, ws, prof);
  return hipErrorInvalidValue;
}

namespace {

template <int NT>
hipError_t launch_batch_terms(hipStream_t st, rid_dtype dtype, const SketchJob *djobs,
                              const int4 *dtab, const int *mts, const int64_t *off,
                              const int64_t *cnt, int nbuckets, int64_t red_off, int64_t red_cnt,
                              const int4 *dsplit, int64_t split_cnt, RidProf *prof) {
  if (split_cnt > 0)
    hipLaunchKernelGGL((bf16_split_grouped<NT>), dim3(static_cast<unsigned>(split_cnt)),
                       dim3(256), 0, st, djobs, dsplit);
  ProfScope ps(prof, st, RID_KERNEL_SKETCH);
  for (int b = 0; b < nbuckets; ++b) {
    if (cnt[b] == 0) continue;
    const dim3 grid(static_cast<unsigned>(cnt[b]));
    const int4 *tb = dtab + off[b];
    // mts[b] counts 16-row tiles of 2l real rows (the bucket key shared by
    // the batch kernels); (mts[b] + 1) / 2 row tiles of Y cover every job of
    // the bucket, and its planes have that many
    switch ((mts[b] + 1) / 2) {
#define RID_BF_CASE(X)                                                                      \
  case X:                                                                                   \
    if (dtype == RID_C64)                                                                   \
      hipLaunchKernelGGL((sketch_bf16_kernel_grouped<X, float2, NT>), grid, dim3(512), 0, st, \
                         djobs, tb);                                                        \
    else                                                                                    \
      hipLaunchKernelGGL((sketch_bf16_kernel_grouped<X, double2, NT>), grid, dim3(512), 0,  \
                         st, djobs, tb);                                                    \
    break;
      RID_BF_CASE(1) RID_BF_CASE(2) RID_BF_CASE(3) RID_BF_CASE(4) RID_BF_CASE(5)
      RID_BF_CASE(6) RID_BF_CASE(7) RID_BF_CASE(8) RID_BF_CASE(9) RID_BF_CASE(10)
      RID_BF_CASE(11) RID_BF_CASE(12) RID_BF_CASE(13) RID_BF_CASE(14)
#undef RID_BF_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  ps.stop();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || red_cnt == 0) return e;
  hipLaunchKernelGGL(bf16_reduce_grouped, dim3(static_cast<unsigned>(red_cnt)), dim3(256), 0, st,
                     djobs, dtab + red_off);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sketch_batch_bf16(hipStream_t st, rid_dtype dtype, int terms,
                                    const SketchJob *djobs, const int4 *dtab, const int *mts,
                                    const int64_t *off, const int64_t *cnt, int nbuckets,
                                    int64_t red_off, int64_t red_cnt, const int4 *dsplit,
                                    int64_t split_cnt, RidProf *prof) {
  if (terms == 2)
    return launch_batch_terms<2>(st, dtype, djobs, dtab, mts, off, cnt, nbuckets, red_off,
                                 red_cnt, dsplit, split_cnt, prof);
  if (terms == 3)
    return launch_batch_terms<3>(st, dtype, djobs, dtab, mts, off, cnt, nbuckets, red_off,
                                 red_cnt, dsplit, split_cnt, prof);
  return hipErrorInvalidValue;
}

template hipError_t launch_sketch_bf16<double2>(hipStream_t, int, int64_t, int64_t, int64_t,
                                                const double2 *, int64_t, const double2 *,
                                                int64_t, double2 *, int64_t, void *, RidProf *);
template hipError_t launch_sketch_bf16<float2>(hipStream_t, int, int64_t, int64_t, int64_t,
                                               const float2 *, int64_t, const double2 *,
                                               int64_t, double2 *, int64_t, void *, RidProf *);
