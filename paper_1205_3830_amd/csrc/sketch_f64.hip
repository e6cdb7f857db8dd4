// sketch_f64.hip -- randomization step Y = G A (Sec. 2) in double precision
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// The complex product is one real GEMM in the real embedding:
//   Yr (2l x n) = Ge (2l x 2m) * Ar (2m x n),
// where Ar is A's memory read as doubles (row 2p = Re A(p,:), row 2p+1 =
// Im A(p,:)), Yr is Y's memory likewise, and the 2x2 block of Ge at (i, p)
// is [[Re g, -Im g], [Im g, Re g]] with g = G(i, p).  Ge is never stored:
// each lane builds its matrix-core operand from the complex G entry.
//
// Tiling (wave64): a workgroup of 4 waves owns 64 columns of A and MT
// 16-row tiles of Yr (all of Yr when 2l <= 16 MT, else a z-slice of them);
// each wave owns 16 of the columns.  One K step covers 16 complex rows of A:
// lane (r16 = lane % 16, q = lane / 16) holds A(p0+4q .. p0+4q+3, column r16)
// -- 64 contiguous bytes, loaded one step ahead -- and the matrix-core k-slot
// q of MFMA number s (s = 0..7) stands for real row 8q + s of the step, so
// the 8 MFMAs of a tile consume those vectors without any shuffle.  The G
// rows of the step (8 MT rows x 16 complex entries) are staged by the whole
// workgroup in LDS, double buffered and loaded one step ahead, with a row
// stride of 17 entries so that the 8 rows read by one MFMA operand fetch
// fall in different banks.  Split-K over m is reduced in a fixed order by a
// second kernel, so the result is deterministic.
#include "rid_internal.hpp"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int MT, class TA>
RID_DEV void sketch_f64_body(
    int64_t m, int64_t n, int64_t l, const TA *__restrict__ A, int64_t lda,
    const double2 *__restrict__ G, int64_t ldg, double *__restrict__ out, int64_t ldo,
    int64_t split_stride, int64_t pchunk, int64_t bx, int64_t by, int64_t bz) {
  constexpr int NR = 8 * MT;                       // G rows of the slab
  constexpr int RS = 17;                           // LDS row stride (complex entries)
  constexpr int PER = (NR * 16 + 255) / 256;       // staged entries per thread
  __shared__ double2 gs[2][NR * RS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int r16 = lane & 15;
  const int c = lane & 1;
  const int64_t jcol = bx * 64 + wave * 16 + r16;
  const bool colok = jcol < n;
  const int64_t pbeg = by * pchunk;
  const int64_t pend = min(m, pbeg + pchunk);
  const int64_t g0 = bz * NR;     // first G row of this z-slice

  d4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  const TA *Acol = A + (colok ? jcol : 0) * lda;
  double2 stg[PER];
  auto load_g = [&](int64_t p0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      const int row = e >> 4, col = e & 15;
      const int64_t i = g0 + row, p = p0 + col;
      stg[r] = (e < NR * 16 && i < l && p < pend) ? G[i * ldg + p] : make_double2(0.0, 0.0);
    }
  };
  auto store_g = [&](int b) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      if (e < NR * 16) gs[b][(e >> 4) * RS + (e & 15)] = stg[r];
    }
  };
  auto load_a = [&](int64_t p0, double2 *a4) {
    const int64_t pb = p0 + 4 * q;
    if (colok && pb + 4 <= pend) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = to_d2(Acol[pb + u]);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        a4[u] = (colok && pb + u < pend) ? to_d2(Acol[pb + u]) : make_double2(0.0, 0.0);
    }
  };

  double2 a4[4], an[4];
  load_g(pbeg);
  store_g(0);
  load_a(pbeg, a4);
  // Wait for the first step's loads here: loads still pending into a4 when
  // the loop starts would make every iteration wait for all outstanding
  // loads -- the next step's prefetch included -- before its first MFMA.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int b = 0;
  for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
    const bool more = p0 + 16 < pend;
    if (more) {
      load_g(p0 + 16);
      load_a(p0 + 16, an);
    }
    const double2 *gb = gs[b];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int row = 8 * t + (r16 >> 1);
      double2 g4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) g4[u] = gb[row * RS + 4 * q + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // row 2i (c = 0): [Re g, -Im g];  row 2i+1 (c = 1): [Im g, Re g]
        const double o0 = c ? g4[u].y : g4[u].x;
        const double o1 = c ? g4[u].x : -g4[u].y;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(o0, a4[u].x, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(o1, a4[u].y, acc[t], 0, 0, 0);
      }
    }
    if (more) {
      store_g(b ^ 1);
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = an[u];
    }
    __syncthreads();
    b ^= 1;
  }
  if (!colok) return;
  // D layout of the f64 16x16x4 MFMA: lane, register r -> row 4r + lane/16,
  // column lane % 16.
  double *o = out + by * split_stride + jcol * ldo;
  const int64_t rows = 2 * l;
  const int64_t mu0 = 2 * g0;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t mu = mu0 + int64_t(t) * 16 + 4 * r + q;
      if (mu < rows) o[mu] = acc[t][r];
    }
}

// One sketch: grid (column blocks, K splits, row slices).
template <int MT, class TA>
__global__ __launch_bounds__(256) void sketch_f64_kernel(
    int64_t m, int64_t n, int64_t l, const TA *__restrict__ A, int64_t lda,
    const double2 *__restrict__ G, int64_t ldg, double *__restrict__ out, int64_t ldo,
    int64_t split_stride, int64_t pchunk) {
  sketch_f64_body<MT, TA>(m, n, l, A, lda, G, ldg, out, ldo, split_stride, pchunk, blockIdx.x,
                          blockIdx.y, blockIdx.z);
}

// A batch: block b runs (job, column block, split) = tab[b] of that job.
template <int MT, class TA>
__global__ __launch_bounds__(256) void sketch_f64_kernel_grouped(const SketchJob *__restrict__ jobs,
                                                     const int4 *__restrict__ tab) {
  const int4 e = tab[blockIdx.x];
  const SketchJob &j = jobs[e.x];
  sketch_f64_body<MT, TA>(j.m, j.n, j.l, static_cast<const TA *>(j.A), j.lda, j.G, j.ldg,
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
  int MT;       // 16-row tiles per block
  int nbz;      // blocks along the Yr rows
  int64_t nbx;  // blocks along columns (64 each)
  int S;        // K splits
  int64_t pchunk;
};

int pick_mt(int64_t tiles) {
  static const int options[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16,
                                18, 20, 22, 24, 26, 28};
  for (int o : options)
    if (o >= tiles) return o;
  return 16;  // more than 28 tiles: several blocks along z, 16 tiles each
}

SketchPlan plan_sketch(int64_t m, int64_t n, int64_t l) {
  SketchPlan p;
  const int64_t tiles = (2 * l + 15) / 16;
  p.MT = pick_mt(tiles);
  p.nbz = static_cast<int>((tiles + p.MT - 1) / p.MT);
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

template <int MT, class TA>
void launch_mt(hipStream_t st, const SketchPlan &p, int64_t m, int64_t n, int64_t l,
               const TA *A, int64_t lda, const double2 *G, int64_t ldg, double *out,
               int64_t ldo, int64_t split_stride) {
  dim3 grid(static_cast<unsigned>(p.nbx), static_cast<unsigned>(p.S),
            static_cast<unsigned>(p.nbz));
  hipLaunchKernelGGL((sketch_f64_kernel<MT, TA>), grid, dim3(256), 0, st, m, n, l, A, lda, G,
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
  switch (p.MT) {
#define RID_MT_CASE(X) \
  case X:              \
    launch_mt<X, TA>(st, p, m, n, l, A, lda, G, ldg, out, ldo, split_stride); \
    break;
    RID_MT_CASE(1) RID_MT_CASE(2) RID_MT_CASE(3) RID_MT_CASE(4) RID_MT_CASE(5)
    RID_MT_CASE(6) RID_MT_CASE(7) RID_MT_CASE(8) RID_MT_CASE(9) RID_MT_CASE(10)
    RID_MT_CASE(11) RID_MT_CASE(12) RID_MT_CASE(13) RID_MT_CASE(14) RID_MT_CASE(15)
    RID_MT_CASE(16) RID_MT_CASE(18) RID_MT_CASE(20) RID_MT_CASE(22) RID_MT_CASE(24)
    RID_MT_CASE(26) RID_MT_CASE(28)
#undef RID_MT_CASE
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
    switch (mts[b]) {
#define RID_MT_CASE(X)                                                                    \
  case X:                                                                                 \
    if (dtype == RID_C64)                                                                 \
      hipLaunchKernelGGL((sketch_f64_kernel_grouped<X, float2>), grid, dim3(256), 0, st, djobs, tb);  \
    else                                                                                  \
      hipLaunchKernelGGL((sketch_f64_kernel_grouped<X, double2>), grid, dim3(256), 0, st, djobs, tb); \
    break;
      RID_MT_CASE(1) RID_MT_CASE(2) RID_MT_CASE(3) RID_MT_CASE(4) RID_MT_CASE(5)
      RID_MT_CASE(6) RID_MT_CASE(7) RID_MT_CASE(8) RID_MT_CASE(9) RID_MT_CASE(10)
      RID_MT_CASE(11) RID_MT_CASE(12) RID_MT_CASE(13) RID_MT_CASE(14) RID_MT_CASE(15)
      RID_MT_CASE(16) RID_MT_CASE(18) RID_MT_CASE(20) RID_MT_CASE(22) RID_MT_CASE(24)
      RID_MT_CASE(26) RID_MT_CASE(28)
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
  int MT, nbz, S;
  int64_t nbx, pchunk, lmax;
};

// lmax: the largest group.  The splits S only grow as lmax shrinks (fewer
// row slices), so lmax = 1 bounds the partials of any grouping.
SrftGemmPlan plan_srft_gemm(int64_t m2, int64_t nb, int64_t lmax) {
  SrftGemmPlan p;
  p.lmax = lmax < 1 ? 1 : lmax;
  const int64_t tiles = (2 * p.lmax + 15) / 16;
  p.MT = pick_mt(tiles);
  p.nbz = static_cast<int>((tiles + p.MT - 1) / p.MT);
  p.nbx = (nb + 63) / 64;
  const int64_t base = p.nbx * p.nbz * 8;
  int64_t S = (4096 + base - 1) / base;
  const int64_t maxS = (m2 + 255) / 256;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  int64_t pchunk = (m2 + S - 1) / S;
  pchunk = (pchunk + 15) / 16 * 16;
  if (pchunk < 16) pchunk = 16;
  if ((m2 + pchunk - 1) / pchunk > 65535) pchunk = ((m2 + 65534) / 65535 + 15) / 16 * 16;
  p.S = static_cast<int>((m2 + pchunk - 1) / pchunk);
  p.pchunk = pchunk;
  return p;
}

struct SrftOff {
  int64_t off[9];
};

template <int MT>
__global__ __launch_bounds__(256) void srft_group_gemm_kernel(
    int64_t m2, int64_t nb, SrftOff g, int nbz, int64_t pchunk, int S,
    const double2 *__restrict__ Z, const double2 *__restrict__ T, double *__restrict__ part) {
  const int t = blockIdx.z / nbz, bz = blockIdx.z % nbz;
  const int64_t lt = g.off[t + 1] - g.off[t];
  if (lt == 0 || int64_t(bz) * 8 * MT >= lt) return;  // uniform over the workgroup
  double *pt = part + int64_t(S) * 2 * nb * g.off[t];
  sketch_f64_body<MT, double2>(m2, nb, lt, Z + int64_t(t) * m2 * nb, m2, T + g.off[t] * m2, m2,
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
    switch (p.MT) {
#define RID_MT_CASE(X)                                                                         \
  case X:                                                                                      \
    hipLaunchKernelGGL((srft_group_gemm_kernel<X>), grid, dim3(256), 0, st, m2, nb, g, p.nbz,  \
                       p.pchunk, p.S, Z, T, part);                                             \
    break;
      RID_MT_CASE(1) RID_MT_CASE(2) RID_MT_CASE(3) RID_MT_CASE(4) RID_MT_CASE(5)
      RID_MT_CASE(6) RID_MT_CASE(7) RID_MT_CASE(8) RID_MT_CASE(9) RID_MT_CASE(10)
      RID_MT_CASE(11) RID_MT_CASE(12) RID_MT_CASE(13) RID_MT_CASE(14) RID_MT_CASE(15)
      RID_MT_CASE(16) RID_MT_CASE(18) RID_MT_CASE(20) RID_MT_CASE(22) RID_MT_CASE(24)
      RID_MT_CASE(26) RID_MT_CASE(28)
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
