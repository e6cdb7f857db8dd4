// sketch_f64.hip -- randomization step Y = G A (Sec. 2) in double precision
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// The complex product is one real GEMM with the embedding on the A side:
//   [Yr Yi] (l x 2n) = [Gr Gi] (l x 2m) * Ae (2m x 2n),
// where [Gr Gi] is G's memory read as doubles (k-index 2p = Re G(:,p),
// 2p+1 = Im G(:,p)), the real column 2j (2j+1) of the result is Re (Im) of
// Y(:,j) -- Y's memory read as doubles -- and the 2x2 block of Ae at (p, j)
// is [[Re a, Im a], [-Im a, Re a]] with a = A(p, j).  Ae is never stored:
// each lane builds its matrix-core operand from the complex A entries it
// loaded, once per K step, and every row tile of the step reuses it; the G
// operand is G's own entries with no rearranging.
//
// Tiling (wave64): a workgroup of 8 waves owns 64 columns of A and RT
// 16-row tiles of Y (all of Y when l <= 16 RT, else a z-slice of them).
// Each wave owns 8 of the columns: real column r16 = lane % 16 of the MFMA
// is part r16 & 1 of complex column r16 >> 1.  One K step covers 16 complex
// rows of A: lane (r16, q = lane/16) holds A(p0+4q .. p0+4q+3, its column)
// -- 64 contiguous bytes, loaded one step ahead -- and the matrix-core
// k-slot q of MFMA number s (s = 0..7) stands for k-index 8q + s of the
// step, i.e. part s & 1 of complex row p0 + 4q + s/2, so the 8 MFMAs of a
// tile consume those vectors without any shuffle.  The G rows of the step
// (16 RT rows x 16 complex entries) are staged by the whole workgroup in
// LDS, double buffered, with a row stride of 17 entries so that the 16 rows
// read by one MFMA operand fetch fall in different banks.  Split-K over m is
// reduced in a fixed order by a second kernel, so the result is
// deterministic.
//
// Against the embedding on the G side (2x2 blocks of G, so that every row
// tile rebuilds its operand with selects and a negation), this takes about
// 40 instead of about 280 vector instructions per step at l = 108, and one
// column group per wave keeps the registers at two waves per SIMD up to
// l = 208.
#include "rid_internal.hpp"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int RT, class TA>
RID_DEV void sketch_f64_body(
    int64_t m, int64_t n, int64_t l, const TA *__restrict__ A, int64_t lda,
    const double2 *__restrict__ G, int64_t ldg, double *__restrict__ out, int64_t ldo,
    int64_t split_stride, int64_t pchunk, int64_t bx, int64_t by, int64_t bz) {
  constexpr int NT = 512;                          // threads per workgroup
  constexpr int KS = 16;                           // complex K rows per step
  constexpr int NR = 16 * RT;                      // G rows of the slab
  constexpr int RS = KS + 1;                       // LDS row stride (complex entries)
  constexpr int PER = (NR * KS + NT - 1) / NT;     // staged entries per thread
  __shared__ double2 gs[2][NR * RS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int r16 = lane & 15;
  const int c = r16 & 1;
  const int64_t jcol = bx * 64 + wave * 8 + (r16 >> 1);
  const bool colok = jcol < n;
  const TA *Acol = A + (colok ? jcol : 0) * lda;
  const int64_t pbeg = by * pchunk;
  const int64_t pend = min(m, pbeg + pchunk);
  const int64_t g0 = bz * NR;     // first G row of this z-slice

  d4 acc[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  auto load_g = [&](int64_t p0, double2 (&stg)[PER]) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + NT * r;
      const int row = e / KS, col = e % KS;
      const int64_t i = g0 + row, p = p0 + col;
      stg[r] = (e < NR * KS && i < l && p < pend) ? G[i * ldg + p] : make_double2(0.0, 0.0);
    }
  };
  auto store_g = [&](int b, const double2 (&stg)[PER]) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + NT * r;
      if (e < NR * KS) gs[b][(e / KS) * RS + (e % KS)] = stg[r];
    }
  };
  // A entries are kept in their stored type until the step that uses them:
  // a conversion right after the load would wait for it there.
  auto load_a = [&](int64_t p0, TA (&v)[4]) {
    const int64_t pb = p0 + 4 * q;
    if (colok && pb + 4 <= pend) {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = Acol[pb + u];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (colok && pb + u < pend) ? Acol[pb + u] : zero_of<TA>();
    }
  };
  // The products of one step: A entries `cur`, G from LDS buffer b.
  auto products = [&](const TA (&cur)[4], int b) {
    // B operand of MFMA s: k-index 2p (s even) carries [Re a, Im a] for
    // parts c = 0, 1; k-index 2p+1 carries [-Im a, Re a]
    double bop[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 v = to_d2(cur[u]);
      bop[2 * u] = c ? v.y : v.x;
      bop[2 * u + 1] = c ? v.x : -v.y;
    }
    const double2 *gb = gs[b];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = 16 * t + r16;
      double2 g4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) g4[u] = gb[row * RS + 4 * q + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(g4[u].x, bop[2 * u], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(g4[u].y, bop[2 * u + 1], acc[t], 0, 0, 0);
      }
    }
  };

  TA a[4], an[4];
  double2 sn[PER];
  load_g(pbeg, sn);
  store_g(0, sn);
  load_a(pbeg, a);
  // Wait for the first step's loads here: loads still pending into `a` when
  // the loop starts would make every iteration wait for all outstanding
  // loads -- the next step's prefetch included -- before its first MFMA.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int b = 0;
  for (int64_t p0 = pbeg; p0 < pend; p0 += KS) {
    const bool more = p0 + KS < pend;
    if (more) {
      load_g(p0 + KS, sn);
      load_a(p0 + KS, an);
    }
    products(a, b);
    if (more) {
      store_g(b ^ 1, sn);
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = an[u];
    }
    __syncthreads();
    b ^= 1;
  }
  if (!colok) return;
  // D layout of the f64 16x16x4 MFMA: lane, register r -> row 4r + lane/16,
  // column lane % 16, here part c of complex column jcol.  `out` holds the
  // real parts of Y's rows at even and the imaginary parts at odd offsets
  // of each column (ldo doubles apart).
  double *o = out + by * split_stride + jcol * ldo;
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = g0 + int64_t(t) * 16 + 4 * r + q;
      if (i < l) o[2 * i + c] = acc[t][r];
    }
}

template <int RT, class TA>
__global__ __launch_bounds__(512) void sketch_f64_kernel(
    int64_t m, int64_t n, int64_t l, const TA *__restrict__ A, int64_t lda,
    const double2 *__restrict__ G, int64_t ldg, double *__restrict__ out, int64_t ldo,
    int64_t split_stride, int64_t pchunk) {
  sketch_f64_body<RT, TA>(m, n, l, A, lda, G, ldg, out, ldo, split_stride, pchunk, blockIdx.x,
                          blockIdx.y, blockIdx.z);
}

// A batch: block b runs (job, column block, split) = tab[b] of that job
// (every job of the launch has l <= 16 RT).
template <int RT, class TA>
__global__ __launch_bounds__(512) void sketch_f64_kernel_grouped(const SketchJob *__restrict__ jobs,
                                                     const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const SketchJob &j = jobs[e.x];
  sketch_f64_body<RT, TA>(j.m, j.n, j.l, static_cast<const TA *>(j.A), j.lda, j.G, j.ldg,
                   static_cast<double *>(j.part), 2 * j.l, 2 * j.l * j.n, j.pchunk, e.y, e.z, 0);
}

// Y(mu, j) = sum over splits s = 0..S-1 (in order) of part[s](mu, j).
__global__ __launch_bounds__(256) void sketch_reduce_kernel(int64_t rows, int64_t n, int S,
                                                            const double *__restrict__ part,
                                                            double *__restrict__ Y,
                                                            int64_t ldy2) {
  const int64_t total = rows * n;
  const int64_t stride = rows * n;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = e / rows;
    const int64_t mu = e - j * rows;
    double s = 0.0;
    for (int sp = 0; sp < S; ++sp) s += part[sp * stride + e];
    Y[j * ldy2 + mu] = s;
  }
}

// A batch of reduces: entry (job, block, blocks of the job).
__global__ __launch_bounds__(256) void sketch_reduce_kernel_grouped(const SketchJob *__restrict__ jobs,
                                                     const int4 *__restrict__ tab) {
  const int4 en = tab[blockIdx.x];
  const SketchJob &jb = jobs[en.x];
  const int64_t rows = 2 * jb.l;
  const int64_t total = rows * jb.n;
  const double *part = static_cast<const double *>(jb.part);
  double *Y = reinterpret_cast<double *>(jb.Y);
  for (int64_t e = int64_t(en.y) * 256 + threadIdx.x; e < total; e += int64_t(en.z) * 256) {
    double s = 0.0;
    for (int64_t sp = 0; sp < jb.S; ++sp) s += static_cast<double>(part[sp * total + e]);
    Y[e] = s;
  }
}

struct SketchPlan {
  int RT;       // 16-row tiles of Y per block
  int nbz;      // blocks along the Yr rows
  int64_t nbx;  // blocks along columns (64 each)
  int S;        // K splits
  int64_t pchunk;
};

// Row tiles per block for `tiles` 16-row tiles of Y: all of them up to 14
// (28 accumulator tiles per wave), else z-slices of 8.
int pick_rt(int64_t tiles) { return tiles <= 14 ? static_cast<int>(tiles < 1 ? 1 : tiles) : 8; }

SketchPlan plan_sketch(int64_t m, int64_t n, int64_t l) {
  SketchPlan p;
  const int64_t tiles = (l + 15) / 16;
  p.RT = pick_rt(tiles);
  p.nbz = static_cast<int>((tiles + p.RT - 1) / p.RT);
  p.nbx = (n + 63) / 64;
  const int64_t base = p.nbx * p.nbz;
  int64_t S = (2048 + base - 1) / base;
  const int64_t maxS = (m + 255) / 256;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  int64_t pchunk = (m + S - 1) / S;
  pchunk = (pchunk + 31) / 32 * 32;  // whole K steps
  if (pchunk < 32) pchunk = 32;
  if (rid_tl_short_blocks && pchunk > RID_SPLIT_ROWS_MAX) pchunk = RID_SPLIT_ROWS_MAX;
  if ((m + pchunk - 1) / pchunk > 65535) pchunk = ((m + 65534) / 65535 + 31) / 32 * 32;  // grid y
  S = (m + pchunk - 1) / pchunk;
  if (S < 1) S = 1;
  p.S = static_cast<int>(S);
  p.pchunk = pchunk;
  return p;
}

template <int RT, class TA>
void launch_rt(hipStream_t st, const SketchPlan &p, int64_t m, int64_t n, int64_t l,
               const TA *A, int64_t lda, const double2 *G, int64_t ldg, double *out,
               int64_t ldo, int64_t split_stride) {
  dim3 grid(static_cast<unsigned>(p.nbx), static_cast<unsigned>(p.S),
            static_cast<unsigned>(p.nbz));
  hipLaunchKernelGGL((sketch_f64_kernel<RT, TA>), grid, dim3(512), 0, st, m, n, l, A, lda, G,
                     ldg, out, ldo, split_stride, p.pchunk);
}

}  // namespace

size_t sketch_f64_ws_bytes(int64_t m, int64_t n, int64_t l) {
  const SketchPlan p = plan_sketch(m, n, l);
  if (p.S <= 1) return 0;
  return size_t(p.S) * size_t(2 * l) * size_t(n) * sizeof(double);
}

template <class TA>
hipError_t launch_sketch_f64(hipStream_t st, int64_t m, int64_t n, int64_t l, const TA *A,
                             int64_t lda, const double2 *G, int64_t ldg, double2 *Y,
                             int64_t ldy, void *partv, RidProf *prof) {
  double *part = static_cast<double *>(partv);
  if (n == 0 || l == 0) return hipSuccess;
  const SketchPlan p = plan_sketch(m, n, l);
  double *out;
  int64_t ldo, split_stride;
  if (p.S <= 1) {
    out = reinterpret_cast<double *>(Y);
    ldo = 2 * ldy;
    split_stride = 0;
  } else {
    out = part;
    ldo = 2 * l;
    split_stride = 2 * l * n;
  }
  ProfScope ps(prof, st, RID_KERNEL_SKETCH);
  switch (p.RT) {
#define RID_RT_CASE(X) \
  case X:              \
    launch_rt<X, TA>(st, p, m, n, l, A, lda, G, ldg, out, ldo, split_stride); \
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
  if (e != hipSuccess || p.S <= 1) return e;
  const int64_t total = 2 * l * n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sketch_reduce_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                     st, 2 * l, n, p.S, part, reinterpret_cast<double *>(Y), 2 * ldy);
  return hipGetLastError();
}

hipError_t launch_sketch_batch_f64(hipStream_t st, rid_dtype dtype, const SketchJob *djobs,
                                     const int4 *dtab, const int *mts, const int64_t *off,
                                     const int64_t *cnt, int nbuckets, int64_t red_off,
                                     int64_t red_cnt, RidProf *prof) {
  ProfScope ps(prof, st, RID_KERNEL_SKETCH);
  for (int b = 0; b < nbuckets; ++b) {
    if (cnt[b] == 0) continue;
    const dim3 grid(static_cast<unsigned>(cnt[b]));
    const int4 *tb = dtab + off[b];
    // mts[b] counts 16-row tiles of the 2l real rows that the FP32 and
    // BF16x3 kernels embed; every job of the bucket has l <= 8 mts[b], so
    // (mts[b] + 1) / 2 row tiles of Y cover it here
    switch ((mts[b] + 1) / 2) {
#define RID_MT_CASE(X)                                                                    \
  case X:                                                                                 \
    if (dtype == RID_C64)                                                                 \
      hipLaunchKernelGGL((sketch_f64_kernel_grouped<X, float2>), grid, dim3(512), 0, st, djobs, tb);  \
    else                                                                                  \
      hipLaunchKernelGGL((sketch_f64_kernel_grouped<X, double2>), grid, dim3(512), 0, st, djobs, tb); \
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
  hipLaunchKernelGGL(sketch_reduce_kernel_grouped, dim3(static_cast<unsigned>(red_cnt)), dim3(256), 0, st, djobs,
                     dtab + red_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------- S F D groups
namespace {

// The block-diagonal product of the four-step S F D sketch: for each residue
// group t < 8 with rows off[t] .. off[t+1]-1 of the grouped order,
//   part_t = T_t Z_t,  T_t = T(off[t] .., :) (l_t x m2, row-major, ld m2),
//   Z_t = Z + t m2 nb (m2 x nb, ld m2),
// split over K like one sketch; grid z runs over (group, row slice).  The
// reduce then writes Y(perm_i[r], j0 + j) = sum of the splits, so the rows
// come back in draw order.
struct SrftGemmPlan {
  int RT, nbz, S;
  int64_t nbx, pchunk, lmax;
};

// lmax: the largest group.  The splits S only grow as lmax shrinks (fewer
// row slices), so lmax = 1 bounds the partials of any grouping.
SrftGemmPlan plan_srft_gemm(int64_t m2, int64_t nb, int64_t lmax) {
  SrftGemmPlan p;
  p.lmax = lmax < 1 ? 1 : lmax;
  const int64_t tiles = (p.lmax + 15) / 16;
  p.RT = pick_rt(tiles);
  p.nbz = static_cast<int>((tiles + p.RT - 1) / p.RT);
  p.nbx = (nb + 63) / 64;
  const int64_t base = p.nbx * p.nbz * 8;
  int64_t S = (4096 + base - 1) / base;
  const int64_t maxS = (m2 + 255) / 256;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  int64_t pchunk = (m2 + S - 1) / S;
  pchunk = (pchunk + 31) / 32 * 32;  // whole K steps
  if (pchunk < 32) pchunk = 32;
  if ((m2 + pchunk - 1) / pchunk > 65535) pchunk = ((m2 + 65534) / 65535 + 31) / 32 * 32;
  p.S = static_cast<int>((m2 + pchunk - 1) / pchunk);
  p.pchunk = pchunk;
  return p;
}

struct SrftOff {
  int64_t off[9];
};

template <int RT>
__global__ __launch_bounds__(512) void srft_group_gemm_kernel(
    int64_t m2, int64_t nb, SrftOff g, int nbz, int64_t pchunk, int S,
    const double2 *__restrict__ Z, const double2 *__restrict__ T, double *__restrict__ part) {
  const int t = blockIdx.z / nbz, bz = blockIdx.z % nbz;
  const int64_t lt = g.off[t + 1] - g.off[t];
  if (lt == 0 || int64_t(bz) * 16 * RT >= lt) return;  // uniform over the workgroup
  double *pt = part + int64_t(S) * 2 * nb * g.off[t];
  sketch_f64_body<RT, double2>(m2, nb, lt, Z + int64_t(t) * m2 * nb, m2, T + g.off[t] * m2, m2,
                               pt, 2 * lt, 2 * lt * nb, pchunk, blockIdx.x, blockIdx.y, bz);
}

__global__ __launch_bounds__(256) void srft_group_reduce_kernel(
    int64_t l, int64_t nb, int64_t j0, SrftOff g, int S, const double *__restrict__ part,
    const int64_t *__restrict__ perm_i, double2 *__restrict__ Y, int64_t ldy) {
  const int64_t total = l * nb;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = e / l, rg = e - j * l;  // grouped row rg of column j
    int t = 0;
    while (t < 7 && rg >= g.off[t + 1]) ++t;
    const int64_t lt = g.off[t + 1] - g.off[t], r = rg - g.off[t];
    const double *pt = part + int64_t(S) * 2 * nb * g.off[t] + j * 2 * lt + 2 * r;
    const int64_t stride = 2 * lt * nb;
    double re = 0.0, im = 0.0;
    for (int sp = 0; sp < S; ++sp) {
      re += pt[sp * stride];
      im += pt[sp * stride + 1];
    }
    const int64_t i = perm_i[rg];
    if (i >= 0 && i < l) Y[(j0 + j) * ldy + i] = make_double2(re, im);
  }
}

}  // namespace

template hipError_t launch_sketch_f64<double2>(hipStream_t, int64_t, int64_t, int64_t,
                                               const double2 *, int64_t, const double2 *,
                                               int64_t, double2 *, int64_t, void *, RidProf *);
template hipError_t launch_sketch_f64<float2>(hipStream_t, int64_t, int64_t, int64_t,
                                              const float2 *, int64_t, const double2 *, int64_t,
                                              double2 *, int64_t, void *, RidProf *);

size_t srft_gemm_ws_bytes(int64_t m2, int64_t nb, int64_t l) {
  const SrftGemmPlan p = plan_srft_gemm(m2, nb, 1);
  return size_t(p.S) * 2 * size_t(nb) * size_t(l) * sizeof(double);
}

hipError_t launch_srft_gemm(hipStream_t st, int64_t m2, int64_t nb, int64_t j0,
                            const int64_t *off, const double2 *Z, const double2 *T,
                            const int64_t *perm_i, double2 *Y, int64_t ldy, void *partv,
                            RidProf *prof) {
  int64_t lmax = 0;
  for (int t = 0; t < 8; ++t) lmax = std::max(lmax, off[t + 1] - off[t]);
  const SrftGemmPlan p = plan_srft_gemm(m2, nb, lmax);
  SrftOff g;
  for (int t = 0; t < 9; ++t) g.off[t] = off[t];
  double *part = static_cast<double *>(partv);
  const dim3 grid(static_cast<unsigned>(p.nbx), static_cast<unsigned>(p.S),
                  static_cast<unsigned>(8 * p.nbz));
  {
    ProfScope ps(prof, st, RID_KERNEL_SKETCH);
    switch (p.RT) {
#define RID_MT_CASE(X)                                                                         \
  case X:                                                                                      \
    hipLaunchKernelGGL((srft_group_gemm_kernel<X>), grid, dim3(512), 0, st, m2, nb, g, p.nbz,  \
                       p.pchunk, p.S, Z, T, part);                                             \
    break;
      RID_MT_CASE(1) RID_MT_CASE(2) RID_MT_CASE(3) RID_MT_CASE(4) RID_MT_CASE(5)
      RID_MT_CASE(6) RID_MT_CASE(7) RID_MT_CASE(8) RID_MT_CASE(9) RID_MT_CASE(10)
      RID_MT_CASE(11) RID_MT_CASE(12) RID_MT_CASE(13) RID_MT_CASE(14)
#undef RID_MT_CASE
      default:
        return hipErrorInvalidValue;
    }
    ps.stop();
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = off[8] * nb;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(srft_group_reduce_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                     st, off[8], nb, j0, g, p.S, part, perm_i, Y, ldy);
  return hipGetLastError();
}
