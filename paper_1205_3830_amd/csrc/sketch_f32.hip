// sketch_f32.hip -- randomization step Y = G A (Sec. 2) with single-precision
// products on the FP32 matrix cores (v_mfma_f32_16x16x4f32), FP32
// accumulation within a K split, and the K splits summed in double into the
// complex128 Y.  The reduced-precision form of the sketch: the pivoted QR,
// the triangular solve and the residual that follow stay in double.
//
// Same real embedding and tiling as the double-precision kernel
// (sketch_f64.hip): [Yr Yi] = [Gr Gi] Ae with the 2x2 blocks [[Re a, Im a],
// [-Im a, Re a]] of Ae built per lane from the A entries it loaded, once per
// K step; a workgroup of 8 waves owns 64 columns of A and RT 16-row tiles of
// Y, each wave 8 of the columns (real column r16 of a tile is part r16 & 1 of
// complex column r16 >> 1); lane (r16, q) holds four consecutive complex
// entries of its column for each 16-row K step and k-slot q of MFMA s stands
// for k-index 8q + s.  G (complex128 in memory) is rounded to complex64 as
// it is staged into LDS, double buffered, row stride 17 entries.  The FP32
// MFMA output layout differs from the FP64 one: lane l, register r holds row
// 4 (l / 16) + r, column l % 16 (measured on gfx950).
#include "rid_internal.hpp"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int RT, class TA>
RID_DEV void sketch_f32_body(
    int64_t m, int64_t n, int64_t l, const TA *__restrict__ A, int64_t lda,
    const double2 *__restrict__ G, int64_t ldg, float *__restrict__ out, int64_t ldo,
    int64_t split_stride, int64_t pchunk, int64_t bx, int64_t by, int64_t bz) {
  constexpr int NT = 512;
  constexpr int NR = 16 * RT;
  constexpr int RS = 17;
  constexpr int PER = (NR * 16 + NT - 1) / NT;
  __shared__ float2 gs[2][NR * RS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int r16 = lane & 15;
  const int c = r16 & 1;
  const int64_t jcol = bx * 64 + wave * 8 + (r16 >> 1);
  const bool colok = jcol < n;
  const int64_t pbeg = by * pchunk;
  const int64_t pend = min(m, pbeg + pchunk);
  const int64_t g0 = bz * NR;

  f4 acc[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  const TA *Acol = A + (colok ? jcol : 0) * lda;
  // Prefetched values stay in their stored type until the end of the step:
  // converting right after a load would make the wave wait for that load
  // there, serialising the prefetch with the step's products.
  double2 stg[PER];
  auto load_g = [&](int64_t p0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + NT * r;
      const int row = e >> 4, col = e & 15;
      const int64_t i = g0 + row, p = p0 + col;
      stg[r] = (e < NR * 16 && i < l && p < pend) ? G[i * ldg + p] : make_double2(0.0, 0.0);
    }
  };
  auto store_g = [&](int b) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + NT * r;
      if (e < NR * 16) gs[b][(e >> 4) * RS + (e & 15)] = to_f2(stg[r]);
    }
  };
  auto load_a = [&](int64_t p0, TA *raw) {
    const int64_t pb = p0 + 4 * q;
    if (colok && pb + 4 <= pend) {
#pragma unroll
      for (int u = 0; u < 4; ++u) raw[u] = Acol[pb + u];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        raw[u] = (colok && pb + u < pend) ? Acol[pb + u] : zero_of<TA>();
    }
  };

  TA a[4], an[4];
  load_g(pbeg);
  store_g(0);
  load_a(pbeg, a);
  // nothing may be pending into `a` when the loop starts (it would make every
  // step wait for its own prefetch before the first product)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int b = 0;
  for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
    const bool more = p0 + 16 < pend;
    // B operand of MFMA s: k-index 2p (s even) carries [Re a, Im a] for
    // parts c = 0, 1; k-index 2p+1 carries [-Im a, Re a]
    float bop[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float2 v = to_f2(a[u]);
      bop[2 * u] = c ? v.y : v.x;
      bop[2 * u + 1] = c ? v.x : -v.y;
    }
    if (more) {
      load_g(p0 + 16);
      load_a(p0 + 16, an);
    }
    const float2 *gb = gs[b];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = 16 * t + r16;
      float2 g4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) g4[u] = gb[row * RS + 4 * q + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(g4[u].x, bop[2 * u], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(g4[u].y, bop[2 * u + 1], acc[t], 0, 0, 0);
      }
    }
    if (more) {
      store_g(b ^ 1);
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = an[u];
    }
    __syncthreads();
    b ^= 1;
  }
  if (!colok) return;
  // `out` holds the real parts of Y's rows at even and the imaginary parts
  // at odd offsets of each column (ldo floats apart)
  float *o = out + by * split_stride + jcol * ldo;
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = g0 + int64_t(t) * 16 + 4 * q + r;
      if (i < l) o[2 * i + c] = acc[t][r];
    }
}

// One sketch: grid (column blocks, K splits, row slices).
template <int RT, class TA>
__global__ __launch_bounds__(512) void sketch_f32_kernel(
    int64_t m, int64_t n, int64_t l, const TA *__restrict__ A, int64_t lda,
    const double2 *__restrict__ G, int64_t ldg, float *__restrict__ out, int64_t ldo,
    int64_t split_stride, int64_t pchunk) {
  sketch_f32_body<RT, TA>(m, n, l, A, lda, G, ldg, out, ldo, split_stride, pchunk, blockIdx.x,
                          blockIdx.y, blockIdx.z);
}

// A batch: block b runs (job, column block, split) = tab[b] of that job
// (every job of the launch has l <= 16 RT).
template <int RT, class TA>
__global__ __launch_bounds__(512) void sketch_f32_kernel_grouped(const SketchJob *__restrict__ jobs,
                                                     const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const SketchJob &j = jobs[e.x];
  sketch_f32_body<RT, TA>(j.m, j.n, j.l, static_cast<const TA *>(j.A), j.lda, j.G, j.ldg,
                   static_cast<float *>(j.part), 2 * j.l, 2 * j.l * j.n, j.pchunk, e.y, e.z, 0);
}

// Y(mu, j) = sum over splits (in order, in double) of part[s](mu, j).
__global__ __launch_bounds__(256) void sketch_f32_reduce_kernel(int64_t rows, int64_t n, int S,
                                                                const float *__restrict__ part,
                                                                double *__restrict__ Y,
                                                                int64_t ldy2) {
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

// A batch of reduces: entry (job, block, blocks of the job).
__global__ __launch_bounds__(256) void sketch_f32_reduce_kernel_grouped(const SketchJob *__restrict__ jobs,
                                                     const int4 *__restrict__ tab) {
  const int4 en = tab[blockIdx.x];
  const SketchJob &jb = jobs[en.x];
  const int64_t rows = 2 * jb.l;
  const int64_t total = rows * jb.n;
  const float *part = static_cast<const float *>(jb.part);
  double *Y = reinterpret_cast<double *>(jb.Y);
  for (int64_t e = int64_t(en.y) * 256 + threadIdx.x; e < total; e += int64_t(en.z) * 256) {
    double s = 0.0;
    for (int64_t sp = 0; sp < jb.S; ++sp) s += static_cast<double>(part[sp * total + e]);
    Y[e] = s;
  }
}

struct Plan32 {
  int RT, nbz;
  int64_t nbx;
  int S;
  int64_t pchunk;
};

int pick_mt32(int64_t tiles) {
  static const int options[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16,
                                18, 20, 22, 24, 26, 28};
  for (int o : options)
    if (o >= tiles) return o;
  return 16;
}

// Row tiles of Y per block for `tiles` 16-row tiles: all of them up to 14,
// else z-slices of 8.
int pick_rt32(int64_t tiles) { return tiles <= 14 ? static_cast<int>(tiles < 1 ? 1 : tiles) : 8; }

Plan32 plan32(int64_t m, int64_t n, int64_t l) {
  Plan32 p;
  const int64_t tiles = (l + 15) / 16;
  p.RT = pick_rt32(tiles);
  p.nbz = static_cast<int>((tiles + p.RT - 1) / p.RT);
  p.nbx = (n + 63) / 64;
  const int64_t base = p.nbx * p.nbz;
  int64_t S = (2048 + base - 1) / base;
  const int64_t maxS = (m + 255) / 256;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  int64_t pchunk = (m + S - 1) / S;
  pchunk = (pchunk + 15) / 16 * 16;
  if (pchunk < 16) pchunk = 16;
  if (rid_tl_short_blocks && pchunk > RID_SPLIT_ROWS_MAX) pchunk = RID_SPLIT_ROWS_MAX;
  if ((m + pchunk - 1) / pchunk > 65535) pchunk = ((m + 65534) / 65535 + 15) / 16 * 16;  // grid y
  S = (m + pchunk - 1) / pchunk;
  if (S < 1) S = 1;
  p.S = static_cast<int>(S);
  p.pchunk = pchunk;
  return p;
}

template <int RT, class TA>
void launch32(hipStream_t st, const Plan32 &p, int64_t m, int64_t n, int64_t l, const TA *A,
              int64_t lda, const double2 *G, int64_t ldg, float *part) {
  dim3 grid(static_cast<unsigned>(p.nbx), static_cast<unsigned>(p.S),
            static_cast<unsigned>(p.nbz));
  hipLaunchKernelGGL((sketch_f32_kernel<RT, TA>), grid, dim3(512), 0, st, m, n, l, A, lda, G,
                     ldg, part, 2 * l, 2 * l * n, p.pchunk);
}

}  // namespace

size_t sketch_f32_ws_bytes(int64_t m, int64_t n, int64_t l) {
  const Plan32 p = plan32(m, n, l);
  return size_t(p.S) * size_t(2 * l) * size_t(n) * sizeof(float);
}

template <class TA>
hipError_t launch_sketch_f32(hipStream_t st, int64_t m, int64_t n, int64_t l, const TA *A,
                             int64_t lda, const double2 *G, int64_t ldg, double2 *Y,
                             int64_t ldy, void *partv, RidProf *prof) {
  if (n == 0 || l == 0) return hipSuccess;
  float *part = static_cast<float *>(partv);
  const Plan32 p = plan32(m, n, l);
  ProfScope ps(prof, st, RID_KERNEL_SKETCH);
  switch (p.RT) {
#define RID_RT_CASE(X) \
  case X:              \
    launch32<X, TA>(st, p, m, n, l, A, lda, G, ldg, part); \
    break;
    RID_RT_CASE(1) RID_RT_CASE(2) RID_RT_CASE(3) RID_RT_CASE(4) RID_RT_CASE(5)
    RID_RT_CASE(6) RID_RT_CASE(7) RID_RT_CASE(8) RID_RT_CASE(9) RID_RT_CASE(10)
    RID_RT_CASE(11) RID_RT_CASE(12) RID_RT_CASE(13) RID_RT_CASE(14)
#undef RID_RT_CASE
    default:
      return hipErrorInvalidValue;
  }
  ps.stop();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = 2 * l * n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sketch_f32_reduce_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                     st, 2 * l, n, p.S, part, reinterpret_cast<double *>(Y), 2 * ldy);
  return hipGetLastError();
}

hipError_t launch_sketch_batch_f32(hipStream_t st, rid_dtype dtype, const SketchJob *djobs,
                                     const int4 *dtab, const int *mts, const int64_t *off,
                                     const int64_t *cnt, int nbuckets, int64_t red_off,
                                     int64_t red_cnt, RidProf *prof) {
  ProfScope ps(prof, st, RID_KERNEL_SKETCH);
  for (int b = 0; b < nbuckets; ++b) {
    if (cnt[b] == 0) continue;
    const dim3 grid(static_cast<unsigned>(cnt[b]));
    const int4 *tb = dtab + off[b];
    // mts[b] counts 16-row tiles of 2l real rows (the bucket key shared by
    // the batch kernels); every job of the bucket has l <= 8 mts[b], so
    // (mts[b] + 1) / 2 row tiles of Y cover it here
    switch ((mts[b] + 1) / 2) {
#define RID_MT_CASE(X)                                                                    \
  case X:                                                                                 \
    if (dtype == RID_C64)                                                                 \
      hipLaunchKernelGGL((sketch_f32_kernel_grouped<X, float2>), grid, dim3(512), 0, st, djobs, tb);  \
    else                                                                                  \
      hipLaunchKernelGGL((sketch_f32_kernel_grouped<X, double2>), grid, dim3(512), 0, st, djobs, tb); \
    break;
      RID_MT_CASE(1) RID_MT_CASE(2) RID_MT_CASE(3) RID_MT_CASE(4) RID_MT_CASE(5)
      RID_MT_CASE(6) RID_MT_CASE(7) RID_MT_CASE(8) RID_MT_CASE(9) RID_MT_CASE(10)
      RID_MT_CASE(11) RID_MT_CASE(12) RID_MT_CASE(13) RID_MT_CASE(14)
#undef RID_MT_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  ps.stop();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || red_cnt == 0) return e;
  hipLaunchKernelGGL(sketch_f32_reduce_kernel_grouped, dim3(static_cast<unsigned>(red_cnt)), dim3(256), 0, st, djobs,
                     dtab + red_off);
  return hipGetLastError();
}

template hipError_t launch_sketch_f32<double2>(hipStream_t, int64_t, int64_t, int64_t,
                                               const double2 *, int64_t, const double2 *,
                                               int64_t, double2 *, int64_t, void *, RidProf *);
template hipError_t launch_sketch_f32<float2>(hipStream_t, int64_t, int64_t, int64_t,
                                              const float2 *, int64_t, const double2 *, int64_t,
                                              double2 *, int64_t, void *, RidProf *);

// ---------------------------------------------------------------- dispatch
hipError_t launch_sketch_batch_f64(hipStream_t st, rid_dtype dtype, const SketchJob *djobs,
                                   const int4 *dtab, const int *mts, const int64_t *off,
                                   const int64_t *cnt, int nbuckets, int64_t red_off,
                                   int64_t red_cnt, RidProf *prof);

hipError_t launch_sketch_batch(hipStream_t st, rid_dtype dtype, rid_prec prec,
                               const SketchJob *djobs, const int4 *dtab, const int *mts,
                               const int64_t *off, const int64_t *cnt, int nbuckets,
                               int64_t red_off, int64_t red_cnt, const int4 *dsplit,
                               int64_t split_cnt, RidProf *prof) {
  if (prec == RID_BF16X2 || prec == RID_BF16X3)
    return launch_sketch_batch_bf16(st, dtype, prec == RID_BF16X2 ? 2 : 3, djobs, dtab, mts, off,
                                    cnt, nbuckets, red_off, red_cnt, dsplit, split_cnt, prof);
  if (prec == RID_FP32)
    return launch_sketch_batch_f32(st, dtype, djobs, dtab, mts, off, cnt, nbuckets, red_off,
                                   red_cnt, prof);
  return launch_sketch_batch_f64(st, dtype, djobs, dtab, mts, off, cnt, nbuckets, red_off,
                                 red_cnt, prof);
}

int sketch_pick_mt(int64_t l) {
  const int64_t tiles = (2 * l + 15) / 16;
  const int mt = pick_mt32(tiles);
  return mt >= tiles ? mt : 0;
}

bool sketch_supported(rid_dtype dtype, rid_prec prec) {
  return (dtype == RID_C128 || dtype == RID_C64) &&
         prec_valid(prec);
}

size_t sketch_ws_bytes(rid_dtype dtype, rid_prec prec, int64_t m, int64_t n, int64_t l) {
  (void)dtype;
  if (prec == RID_BF16X2 || prec == RID_BF16X3) return sketch_bf16_ws_bytes(m, n, l);
  return prec == RID_FP32 ? sketch_f32_ws_bytes(m, n, l) : sketch_f64_ws_bytes(m, n, l);
}

hipError_t launch_sketch(hipStream_t st, rid_dtype dtype, rid_prec prec, int64_t m, int64_t n,
                         int64_t l, const void *A, int64_t lda, const double2 *G, int64_t ldg,
                         double2 *Y, int64_t ldy, void *part, RidProf *prof) {
  if (prec == RID_BF16X2 || prec == RID_BF16X3) {
    const int terms = prec == RID_BF16X2 ? 2 : 3;
    if (dtype == RID_C64)
      return launch_sketch_bf16(st, terms, m, n, l, static_cast<const float2 *>(A), lda, G, ldg,
                                Y, ldy, part, prof);
    return launch_sketch_bf16(st, terms, m, n, l, static_cast<const double2 *>(A), lda, G, ldg,
                              Y, ldy, part, prof);
  }
  if (prec == RID_FP32) {
    if (dtype == RID_C64)
      return launch_sketch_f32(st, m, n, l, static_cast<const float2 *>(A), lda, G, ldg, Y, ldy,
                               part, prof);
    return launch_sketch_f32(st, m, n, l, static_cast<const double2 *>(A), lda, G, ldg, Y, ldy,
                             part, prof);
  }
  if (dtype == RID_C64)
    return launch_sketch_f64(st, m, n, l, static_cast<const float2 *>(A), lda, G, ldg, Y, ldy,
                             part, prof);
  return launch_sketch_f64(st, m, n, l, static_cast<const double2 *>(A), lda, G, ldg, Y, ldy,
                           part, prof);
}
