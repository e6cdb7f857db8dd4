// rid_internal.hpp -- declarations shared by the librid translation units:
// the handle, workspace carving, device helpers (Philox draws, compensated
// double-double arithmetic, wave64 reductions) and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <vector>

#include "rid.h"

// ------------------------------------------------------------------ profiling
// Event pairs recorded around launches of the hot kernels (rid_profile).
struct RidProf {
  bool on = false;
  std::vector<hipEvent_t> pool;              // created events, reused
  size_t used = 0;                           // events handed out since enable
  std::vector<std::pair<int, size_t>> recs;  // (kernel family, index of start event)
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

// Records the start event in the constructor and the stop event in stop();
// a no-op when profiling is off or prof is null.
struct ProfScope {
  RidProf *p;
  hipStream_t st;
  size_t idx = 0;
  bool active = false;
  ProfScope(RidProf *prof, hipStream_t s, int kernel) : p(prof), st(s) {
    if (p && p->on) {
      idx = p->used;
      hipEvent_t a = p->next();
      hipEvent_t b = p->next();
      if (a && b && hipEventRecord(a, st) == hipSuccess) {
        p->recs.emplace_back(kernel, idx);
        active = true;
      }
    }
  }
  void stop() {
    if (active) {
      (void)hipEventRecord(p->pool[idx + 1], st);
      active = false;
    }
  }
  ~ProfScope() { stop(); }
};

// ------------------------------------------------------------------ handle
struct rid_ctx {
  int device = 0;
  int last_hip_error = 0;
  int *d_status = nullptr;  // device status word (RID_OK / RID_ERR_RANK)
  void *ws = nullptr;       // grow-only workspace
  size_t ws_bytes = 0;
  std::vector<void *> retired;  // superseded workspaces, freed by rid_destroy
  size_t retired_bytes = 0;     // their total size
  RidProf prof;
  int sketch_kind = RID_SKETCH_GAUSSIAN;  // operator drawn by rid_sketch / rid_decompose
  int qr_kind = RID_QR_HOUSEHOLDER;       // method of rid_pivqr / rid_decompose
  int residual_kind = RID_RESIDUAL_AUTO;  // accumulation of the residual (rid_set_residual)
  hipStream_t cap_stream = nullptr;       // stream used to capture batch graphs
  bool batch_graph = true;                // capture batches into a graph (else launch directly)
  // plan of the batched path (rid_set_batch_plan / rid_tune_batched)
  int64_t batch_sketch_rows = 1024;       // rows of A per sketch K split
  int64_t batch_res_block_bytes = 256 << 10;  // bytes of A per ax workgroup
  int batch_ahz_cpw = 8;                  // columns per wave of the ahz pass (4 or 8)
};

// Bump allocator over the handle workspace (256-byte aligned pieces).
struct WsCarve {
  char *base;
  size_t off = 0;
  explicit WsCarve(void *b) : base(static_cast<char *>(b)) {}
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
  // the byte offset of the next piece (for layouts computed before the base
  // address is known)
  template <class T>
  size_t take_off(size_t count) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += count * sizeof(T);
    return o;
  }
};

// ------------------------------------------------------------------ device helpers
#define RID_DEV __device__ __forceinline__

// Philox4x32-10 block (Salmon et al., SC'11).
RID_DEV void rid_philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0];
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

RID_DEV double rid_u52(uint32_t lo, uint32_t hi) {
  const uint64_t x = ((static_cast<uint64_t>(hi) << 32) | lo) >> 12;
  return static_cast<double>(2 * x + 1) * 0x1p-53;
}

// One complex Gaussian (Re, Im ~ N(0, 1/2)) of the project's stream:
// counter (col lo, col hi, row, stream), key (seed lo, seed hi), polar
// Box-Muller g = sqrt(-ln u1) e^{2 pi i u2}.
RID_DEV double2 rid_gauss(uint64_t seed, uint32_t stream, uint32_t row, uint64_t col) {
  uint32_t c[4] = {static_cast<uint32_t>(col), static_cast<uint32_t>(col >> 32), row, stream};
  rid_philox10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const double u1 = rid_u52(c[0], c[1]);
  const double u2 = rid_u52(c[2], c[3]);
  const double rad = sqrt(-log(u1));
  const double ang = 6.283185307179586476925286766559 * u2;
  return make_double2(rad * cos(ang), rad * sin(ang));
}

// The first uniform of Philox counter (col lo, col hi, 0, stream): the draws
// of the S F D operator (phases: stream 5, rows: stream 6).
RID_DEV double rid_u1(uint64_t seed, uint32_t stream, uint64_t col) {
  uint32_t c[4] = {static_cast<uint32_t>(col), static_cast<uint32_t>(col >> 32), 0u, stream};
  rid_philox10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  return rid_u52(c[0], c[1]);
}

// Streaming load of one complex128 that is read once per pass (non-temporal:
// it does not displace cached data such as the vectors the pass reuses).
typedef double rid_dv2 __attribute__((ext_vector_type(2)));
RID_DEV double2 ld_stream(const double2 *p) {
  const rid_dv2 v = __builtin_nontemporal_load(reinterpret_cast<const rid_dv2 *>(p));
  return make_double2(v.x, v.y);
}

// complex64 streaming load, widened to double
typedef float rid_fv2 __attribute__((ext_vector_type(2)));
RID_DEV double2 ld_stream(const float2 *p) {
  const rid_fv2 v = __builtin_nontemporal_load(reinterpret_cast<const rid_fv2 *>(p));
  return make_double2(static_cast<double>(v.x), static_cast<double>(v.y));
}

// two adjacent complex64 entries in one 16-byte non-temporal load (p must be
// 16-byte aligned)
typedef float rid_fv4 __attribute__((ext_vector_type(4)));
RID_DEV void ld_stream_pair(const float2 *p, double2 &a, double2 &b) {
  const rid_fv4 v = __builtin_nontemporal_load(reinterpret_cast<const rid_fv4 *>(p));
  a = make_double2(static_cast<double>(v.x), static_cast<double>(v.y));
  b = make_double2(static_cast<double>(v.z), static_cast<double>(v.w));
}

// A raw buffer resource over the given bytes: loads past the end read zeros
// and stores past it are dropped by the hardware's range check, so a column
// slice needs no per-row predicates (and an empty one no branch).  Word 3 is
// the 32-bit data format that every gfx9 target takes.  Buffer loads count
// only against the vector-memory counter, so waiting for an LDS access does
// not also wait for them (as it would for a flat load).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
RID_DEV __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, bytes, 0x00020000);
}
RID_DEV double2 buf_ld(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
RID_DEV void buf_st(__amdgpu_buffer_rsrc_t r, int off, double2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 0);
}

// A value that is the same in every lane but that the compiler cannot see
// as such (read from LDS), made explicitly uniform.
RID_DEV int64_t uniform_i64(int64_t v) {
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32));
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<int>(v));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
RID_DEV double uniform_f64(double v) {
  return __builtin_bit_cast(double, uniform_i64(__builtin_bit_cast(int64_t, v)));
}

// p[i] where the index is the same in every lane and no kernel writes p
// while this one runs: read through the constant address space, so that the
// load is one scalar load (the scalar cache starts each kernel invalidated)
// instead of a vector load that every lane repeats.
RID_DEV double2 ld_uniform(const double2 *p, int64_t i) {
  const __attribute__((address_space(4))) double *q =
      (const __attribute__((address_space(4))) double *)p;
  return make_double2(q[2 * i], q[2 * i + 1]);
}

template <class T>
RID_DEV T zero_of();
template <>
RID_DEV double2 zero_of<double2>() {
  return make_double2(0.0, 0.0);
}
template <>
RID_DEV float2 zero_of<float2>() {
  return make_float2(0.0f, 0.0f);
}

RID_DEV double2 to_d2(double2 v) { return v; }
RID_DEV double2 to_d2(float2 v) {
  return make_double2(static_cast<double>(v.x), static_cast<double>(v.y));
}
RID_DEV float2 to_f2(double2 v) {
  return make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}
RID_DEV float2 to_f2(float2 v) { return v; }

// Error-free transformations (Knuth TwoSum; TwoProd through FMA).  Each
// helper turns off FMA contraction: fusing the product a*b into a following
// sum would make the rounded product and its error term disagree.
RID_DEV void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// s + c += a * b, compensated (one step of Ogita-Rump-Oishi Dot2).
RID_DEV void dot2_acc(double &s, double &c, double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  const double pe = fma(a, b, -p);
  double t, se;
  two_sum(s, p, t, se);
  s = t;
  c += se + pe;
}

// (s1, c1) += (s2, c2) for unnormalised double-double pairs.
RID_DEV void dd_add(double &s1, double &c1, double s2, double c2) {
#pragma clang fp contract(off)
  double t, e;
  two_sum(s1, s2, t, e);
  s1 = t;
  c1 = c1 + c2 + e;
}

// Normalise (s, c) to hi + lo with |lo| <= ulp(hi)/2.
RID_DEV void dd_norm(double s, double c, double &hi, double &lo) {
#pragma clang fp contract(off)
  hi = s + c;
  lo = c - (hi - s);
}

// The value of lane (lane op CTRL) for a DPP lane pattern CTRL, as two
// 32-bit DPP moves: a VALU operation, where a shuffle goes through the LDS
// unit and waits for it.
template <int CTRL>
RID_DEV double dpp_f64(double v) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_update_dpp(0u, static_cast<unsigned>(u), CTRL, 0xF, 0xF,
                                                  false);
  const unsigned hi = __builtin_amdgcn_update_dpp(0u, static_cast<unsigned>(u >> 32), CTRL, 0xF,
                                                  0xF, false);
  return __longlong_as_double((static_cast<unsigned long long>(hi) << 32) | lo);
}

// A 64-bit value of lane (lane op CTRL), moved as bits.
template <int CTRL>
RID_DEV int64_t dpp_i64(int64_t v) {
  return __builtin_bit_cast(int64_t, dpp_f64<CTRL>(__builtin_bit_cast(double, v)));
}

// The gfx950 lane-swap instructions (W = 32: lane ^ 32, W = 16: lane ^ 16)
// applied to a register and its own copy: x and y get, in each lane, its
// own value in one and the partner lane's in the other.  Which is which
// depends on the lane, and is the same for every register swapped, so a
// symmetric combination of x and y (a sum, a maximum) is the butterfly step.
template <int W>
RID_DEV void swap_pair(double v, double &x, double &y) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = static_cast<unsigned>(u), hi = static_cast<unsigned>(u >> 32);
  const auto a = (W == 32) ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                           : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = (W == 32) ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                           : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  x = __longlong_as_double((static_cast<unsigned long long>(b[0]) << 32) | a[0]);
  y = __longlong_as_double((static_cast<unsigned long long>(b[1]) << 32) | a[1]);
}
template <int W>
RID_DEV void swap_pair(int64_t v, int64_t &x, int64_t &y) {
  double dx, dy;
  swap_pair<W>(__builtin_bit_cast(double, v), dx, dy);
  x = __builtin_bit_cast(int64_t, dx);
  y = __builtin_bit_cast(int64_t, dy);
}

// v plus the value of lane ^ W (W = 32 or 16); the same bits in both lanes.
template <int W>
RID_DEV double swap_add(double v) {
  double x, y;
  swap_pair<W>(v, x, y);
  return x + y;
}

// v of lane src (src the same in every lane; that lane active), read into
// scalar registers: no trip through the LDS unit as a shuffle would take.
RID_DEV double lane_bcast(double v, int src) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(static_cast<int>(u), src);
  const unsigned hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), src);
  return __longlong_as_double((static_cast<unsigned long long>(hi) << 32) | lo);
}

// Sum over the 64 lanes of a wave (all active), every lane getting the same
// bits: the butterfly over lane bits 5, 4, ..., 0, each level adding the
// partner lane's value.  Bits 5 and 4 go through the lane-swap instructions
// and bit 3 through a rotation of each 16-lane row by 8 (the same exchange).
// From there on a lane's value depends only on its lane index mod 8, mod 4,
// mod 2, so a row rotation by 4 and the quad patterns [2,3,0,1], [1,0,3,2]
// read a lane that holds the partner's value.  Nothing goes through the LDS
// unit, which the wave's other work keeps busy.
RID_DEV double wave_sum(double v) {
  v = swap_add<32>(v);
  v = swap_add<16>(v);
  v += dpp_f64<0x128>(v);  // row_ror:8
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  return v;
}

// Double-double wave sum (all 64 lanes active), the butterfly of wave_sum:
// dd_add gives the same bits whichever pair comes first, so every lane
// ends with the same (s, c).
template <int CTRL>
RID_DEV void dd_add_dpp(double &s, double &c) {
  const double s2 = dpp_f64<CTRL>(s), c2 = dpp_f64<CTRL>(c);
  dd_add(s, c, s2, c2);
}
template <int W>
RID_DEV void dd_add_swap(double &s, double &c) {
  double s1, s2, c1, c2;
  swap_pair<W>(s, s1, s2);
  swap_pair<W>(c, c1, c2);
  dd_add(s1, c1, s2, c2);
  s = s1;
  c = c1;
}
RID_DEV void wave_sum_dd(double &s, double &c) {
  dd_add_swap<32>(s, c);
  dd_add_swap<16>(s, c);
  dd_add_dpp<0x128>(s, c);  // row_ror:8
  dd_add_dpp<0x124>(s, c);  // row_ror:4
  dd_add_dpp<0x4E>(s, c);   // quad_perm [2,3,0,1]
  dd_add_dpp<0xB1>(s, c);   // quad_perm [1,0,3,2]
}

// Sums NV double-double values (s[v], c[v]) (NV a power of two, 2..64) over
// the 64 lanes of a wave by reduce-scatter: at the level of lane bit b (from
// bit 5 down) each lane keeps the half of its values that the bit selects
// and adds the partner's copy of that half, so after log2(NV) levels a lane
// holds one value, v = lane >> (6 - log2(NV)); the remaining lane bits
// finish it with a plain butterfly.  For NV = 16 that is 34 double shuffles
// and 17 compensated adds, against 192 and 96 for 16 separate wave sums.  On
// return (s[0], c[0]) of every lane is the total of its value v (dd_add is
// symmetric, so all lanes of a group hold the same bits).
// One level of wave_reduce_dd (HALF values kept of 2 HALF), then the next;
// a compile-time recursion, so that every index into s and c is a constant
// (an index the compiler cannot resolve becomes a chain of compares and
// selects over the whole array).
template <int NV, int HALF>
RID_DEV void wave_reduce_dd_level(double (&s)[NV], double (&c)[NV], int lane) {
  if constexpr (HALF >= 1) {
    constexpr int off = HALF * (64 / NV);
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int j = 0; j < HALF; ++j) {
      double ks = up ? s[HALF + j] : s[j], kc = up ? c[HALF + j] : c[j];
      const double gs = __shfl_xor(up ? s[j] : s[HALF + j], off, 64);
      const double gc = __shfl_xor(up ? c[j] : c[HALF + j], off, 64);
      dd_add(ks, kc, gs, gc);
      s[j] = ks;
      c[j] = kc;
    }
    wave_reduce_dd_level<NV, HALF / 2>(s, c, lane);
  }
}

template <int NV>
RID_DEV void wave_reduce_dd(double (&s)[NV], double (&c)[NV]) {
  static_assert(NV >= 2 && NV <= 64 && (NV & (NV - 1)) == 0, "NV: power of two in 2..64");
  const int lane = threadIdx.x & 63;
  constexpr int GROUP = 64 / NV;  // lanes that end up holding the same value
  wave_reduce_dd_level<NV, NV / 2>(s, c, lane);
#pragma unroll
  for (int off = GROUP / 2; off >= 1; off >>= 1) {
    const double gs = __shfl_xor(s[0], off, 64);
    const double gc = __shfl_xor(c[0], off, 64);
    dd_add(s[0], c[0], gs, gc);
  }
}

// ------------------------------------------------------------------ plans
// Short-workgroup plans for a shared device.  When the calling thread has
// rid_tl_short_blocks set (the serving lanes set it for themselves), the
// A-streaming kernels bound the work of one workgroup (rows of a sketch K
// split; columns of an ax split) so that a workgroup lives about a
// millisecond and the dispatcher can hand freed CU slots to kernels of other
// streams (a served batch beside a big ID) instead of making them wait out a
// whole pass.  It costs a few percent more partial sums, so a plain call
// keeps the long-workgroup plans.  Workspace sizing and launches read the
// flag on the same thread within one call, so they always agree.
constexpr int64_t RID_SPLIT_ROWS_MAX = 4096;
constexpr int64_t RID_AX_COLS_MAX = 512;
extern thread_local bool rid_tl_short_blocks;

// ------------------------------------------------------------------ batches
// One job of a batch as the library sees it (device pointers for data).
struct RidBatchJob {
  int64_t m, n, k, l, lda, ldp;
  const void *A;
  uint64_t seed;
  int64_t *J;
  double2 *P;
  double *sigma;
};

// One sketch of a batch (device pointers).  part holds S x 2l x n partial
// sums (double for FP64 products, float for FP32); Y is l x n, ldy = l.
struct SketchJob {
  int64_t m, n, l, lda, ldg, pchunk;
  const void *A;
  const double2 *G;
  void *part;
  double2 *Y;
  int64_t S;
  int64_t red_blocks;  // blocks of the reduce for this job
  // bfloat16-split products only: the split planes of [Gr Gi] (bf16, plane
  // s at s * pstride, entry (i, kappa) at i * ldk + kappa, prow x ldk each)
  void *planes;
  int64_t ldk, pstride, prow;
};

// One interpolation of a batch: R (k x n, ldr), J (k), P (k x n, ldp), and
// mark[j] = t if column j is J[t], -1 otherwise.
struct InterpJob {
  int64_t n, k, ldr, ldp;
  const double2 *R;
  const int64_t *J;
  double2 *P;
  const int *mark;
};

// One pivoted QR of a batch: Y (l x n, ldy) is overwritten by R, J gets the
// k pivots, mark[j] the step at which column j was picked (-1 otherwise);
// the rest is per-job workspace (pivqr_job_ws_bytes).
struct PivJob {
  int64_t l, n, k, ldy;
  double2 *Y;
  int64_t *J;
  int *mark;
  int *status;
  double rank_tol;
  double *cnorm, *cnorm2;
  int64_t *cidx;
  double2 *ccol;
  double *nu0;
};

// Host-side description of a grouped launch sequence: per-job descriptors
// (opaque bytes, copied to the device as an array) and, per step, a table of
// (job, block x, block y) entries, concatenated.
struct GroupedHost {
  std::vector<char> jobs;
  std::vector<int4> tab;
  int64_t off[16];
  int64_t cnt[16];
  size_t ws_bytes = 0;
};

// ------------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error.  Sizes are validated by the
// caller (api.hip); the kernels bound-check every access themselves.

// rows x cols complex128 block (column-major, ld) set to zero.
hipError_t launch_zero(hipStream_t st, int64_t rows, int64_t cols, double2 *out, int64_t ld);

hipError_t launch_gaussian(hipStream_t st, int64_t rows, int64_t cols, uint64_t seed,
                           uint32_t stream_id, double2 *out, int64_t ld);

// rows x m block of the subsampled randomized Fourier operator S F D
// (row-major, ld); requires m < 2^31.
hipError_t launch_srft(hipStream_t st, int64_t rows, int64_t m, uint64_t seed, double2 *out,
                       int64_t ld);

// The sketch operator of the handle's kind (rows = l, cols = m).
hipError_t launch_operator(hipStream_t st, int kind, int64_t rows, int64_t cols, uint64_t seed,
                           double2 *out, int64_t ld);

// Y = S F D A through the four-step DFT (FP64 products; m a multiple of 8,
// l <= 2048): draws as launch_srft's, ws of srft_sketch_ws_bytes bytes.
bool srft_fft_ok(rid_prec prec, int64_t m, int64_t l);
// Its block-diagonal product (sketch_f64.hip): off[0..8] are the row offsets
// of the 8 residue groups in the grouped order (off[8] = l); Z holds the 8
// planes Z_t (m2 x nb each), T the grouped twiddle rows (l x m2); the result
// goes to Y(perm_i[r], j0 + j), rows back in draw order.
size_t srft_gemm_ws_bytes(int64_t m2, int64_t nb, int64_t l);  // any grouping of l rows
hipError_t launch_srft_gemm(hipStream_t st, int64_t m2, int64_t nb, int64_t j0,
                            const int64_t *off, const double2 *Z, const double2 *T,
                            const int64_t *perm_i, double2 *Y, int64_t ldy, void *part,
                            RidProf *prof);
size_t srft_sketch_ws_bytes(int64_t m, int64_t n, int64_t l);
hipError_t launch_srft_sketch(hipStream_t st, rid_dtype dtype, int64_t m, int64_t n, int64_t l,
                              const void *A, int64_t lda, uint64_t seed, double2 *Y, int64_t ldy,
                              void *ws, RidProf *prof);

// Y (complex128) = G A, G complex128 row-major (l x m, ldg), A column-major
// (m x n, lda) of storage type `dtype`, products in precision `prec`.
// part: workspace of sketch_ws_bytes(...) bytes.
bool sketch_supported(rid_dtype dtype, rid_prec prec);
size_t sketch_ws_bytes(rid_dtype dtype, rid_prec prec, int64_t m, int64_t n, int64_t l);
hipError_t launch_sketch(hipStream_t st, rid_dtype dtype, rid_prec prec, int64_t m, int64_t n,
                         int64_t l, const void *A, int64_t lda, const double2 *G, int64_t ldg,
                         double2 *Y, int64_t ldy, void *part, RidProf *prof);

// Grouped sketch over a batch: for each MT bucket the (job, bx, split)
// table slice, then the grouped reduce over (job, block, blocks-of-job).
// The bfloat16-split products first split each job's G into its planes, one
// workgroup per (job, block, blocks-of-job) entry of dsplit (split_cnt
// entries), and take 128 columns per bx instead of 64.
hipError_t launch_sketch_batch(hipStream_t st, rid_dtype dtype, rid_prec prec,
                               const SketchJob *djobs, const int4 *dtab, const int *mts,
                               const int64_t *off, const int64_t *cnt, int nbuckets,
                               int64_t red_off, int64_t red_cnt, const int4 *dsplit,
                               int64_t split_cnt, RidProf *prof);
hipError_t launch_sketch_batch_bf16(hipStream_t st, rid_dtype dtype, int terms,
                                    const SketchJob *djobs, const int4 *dtab, const int *mts,
                                    const int64_t *off, const int64_t *cnt, int nbuckets,
                                    int64_t red_off, int64_t red_cnt, const int4 *dsplit,
                                    int64_t split_cnt, RidProf *prof);
// Columns of A per sketch workgroup of a batch job (64, or 128 for the
// bfloat16-split products).
inline int64_t sketch_batch_cols(rid_prec prec) {
  return prec == RID_BF16X2 || prec == RID_BF16X3 ? 128 : 64;
}
int sketch_pick_mt(int64_t l);  // tiles per block for one batch job (0: unsupported)

bool batch_job_supported(const RidBatchJob &j);
bool batch_prec_supported(rid_prec prec);
// Make the handle's workspace at least `bytes` long.  A larger buffer
// (>= 1.5x the old one) replaces the old, which is kept until rid_destroy:
// work still in flight may use it, and growing never waits for the device
// (hipFree would wait for every stream, other callers' included).
hipError_t grow_ws(rid_handle h, size_t bytes);
// The bytes grow_ws(h, bytes) would allocate (0 when the workspace is large
// enough already); at most that, as grow_ws may fall back to the exact size.
size_t ws_grow_bytes(const rid_ctx *h, size_t bytes);
// Device memory the handle's workspaces hold: the current one and the
// superseded ones.
size_t ws_held_bytes(const rid_ctx *h);
// Free the handle's workspaces (hipFree: waits for the whole device).  Only
// for a handle with no work in flight; the next call grows it again.
void release_ws(rid_handle h);
// Device workspace rid_decompose needs for one ID of this shape.
size_t decomp_ws_bytes(rid_dtype dt, rid_prec pr, int64_t m, int64_t n, int64_t k, int64_t l,
                       int q);
// prof non-null: launch directly (no graph) and time the kernel families into prof.
hipError_t run_batch(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                     const RidBatchJob *bj, int count, int q, double rank_tol, int *status,
                     RidProf *prof = nullptr);
// The workspace bytes run_batch needs for these jobs under the handle's plan
// (host planning only: no device call; the jobs' A, lda and outputs are not
// read).  A subset of the jobs needs no more.
size_t batch_ws_need(rid_handle h, rid_dtype dtype, rid_prec prec, const RidBatchJob *bj,
                     int count, int q);

// Grouped interpolation (k <= 256): tab entries (job, column group of
// interp_blocks).
hipError_t launch_interp_batch(hipStream_t st, int kmax, const InterpJob *djobs,
                               const int4 *dtab, int64_t count, RidProf *prof);

// per-precision launchers behind launch_sketch
size_t sketch_f64_ws_bytes(int64_t m, int64_t n, int64_t l);
template <class TA>
hipError_t launch_sketch_f64(hipStream_t st, int64_t m, int64_t n, int64_t l, const TA *A,
                             int64_t lda, const double2 *G, int64_t ldg, double2 *Y,
                             int64_t ldy, void *part, RidProf *prof);
size_t sketch_bf16_ws_bytes(int64_t m, int64_t n, int64_t l);
// terms: 2 (RID_BF16X2) or 3 (RID_BF16X3) bf16 terms per operand
template <class TA>
hipError_t launch_sketch_bf16(hipStream_t st, int terms, int64_t m, int64_t n, int64_t l,
                              const TA *A, int64_t lda, const double2 *G, int64_t ldg,
                              double2 *Y, int64_t ldy, void *ws, RidProf *prof);

// A product arithmetic this library knows (rid_prec).
inline bool prec_valid(int prec) { return prec >= RID_FP64 && prec <= RID_BF16X3; }
size_t sketch_f32_ws_bytes(int64_t m, int64_t n, int64_t l);
template <class TA>
hipError_t launch_sketch_f32(hipStream_t st, int64_t m, int64_t n, int64_t l, const TA *A,
                             int64_t lda, const double2 *G, int64_t ldg, double2 *Y,
                             int64_t ldy, void *part, RidProf *prof);

// Pivoted QR workspace and launch.
// kind: RID_QR_HOUSEHOLDER or RID_QR_CGS2 (k <= 1024).
size_t pivqr_ws_bytes(int64_t l, int64_t n, int64_t k, int kind);
bool pivqr_supported(int64_t l);
hipError_t launch_pivqr(hipStream_t st, int64_t l, int64_t n, int64_t k, double2 *Y,
                        int64_t ldy, int64_t *perm, double *gaps, double rank_tol,
                        void *ws, int *d_status, RidProf *prof, int kind);

// Batched pivoted QR: one grouped launch per step over the (job, column
// block, blocks of job) table; every job's table entries are its
// pivqr_blocks(n) column blocks.
int64_t pivqr_blocks(int64_t n);
size_t pivqr_job_ws_bytes(int64_t l, int64_t n);
void pivqr_job_carve(char *base, PivJob &jb);
// The QR of every job of a batch in one launch, one workgroup per job, jobs
// in the order given (device array of count job indices).
hipError_t launch_pivqr_jobs(hipStream_t st, const PivJob *djobs, const int *dorder, int count,
                             RidProf *prof);
// One grouped launch per step t = 0 .. kmax: the first live[t] entries of
// the table (the jobs with k >= t come first), lmax[t] their largest l.
hipError_t launch_pivqr_batch(hipStream_t st, const int64_t *lmax, const int64_t *live,
                              int64_t kmax, const PivJob *djobs, const int4 *dtab, int64_t count,
                              RidProf *prof, int cb);

// SVD of A(:, J) P (k <= 256): workspace size and launch.  Synchronises the
// stream (to read the sweep count and the breakdown flag); *rank_bad is set
// when one of the two CholeskyQR3 runs breaks down.
bool svd_supported(int64_t k);
size_t svd_ws_bytes(int64_t m, int64_t n, int64_t k);
hipError_t launch_svd(hipStream_t st, rid_dtype dtype, int64_t m, int64_t n, int64_t k,
                      const void *A, int64_t lda, const int64_t *J, const double2 *P, int64_t ldp,
                      double2 *U, int64_t ldu, double *S, double2 *V, int64_t ldv, void *ws,
                      int *rank_bad, int *sweeps_used);

size_t interp_ws_bytes(int64_t n, int64_t k);
bool interp_supported(int64_t k);
// Workgroups of the direct solve (k <= 256) for n columns of P.
int64_t interp_blocks(int64_t n);
hipError_t launch_interp(hipStream_t st, int64_t n, int64_t k, const double2 *R, int64_t ldr,
                         const int64_t *J, double2 *P, int64_t ldp, void *ws,
                         RidProf *prof);

// Grouped power iteration over a batch: setup on the host (ws == nullptr
// only sizes the workspace), then one launch per step for all jobs.
// Accumulation of the residual's passes over A.
enum ResAcc : int {
  RES_DOT2 = 0,  // compensated (double-double) sums
  RES_FP64 = 1,  // plain double FMA chains
  RES_FP32 = 2   // single-precision products and sums per slab, partials in double
};

// The accumulation a handle's residual takes for sketch arithmetic `prec`
// (rid_set_residual; automatic: compensated for RID_FP64, plain double for
// the reduced-precision forms).
inline int res_acc(int residual_kind, int prec) {
  switch (residual_kind) {
    case RID_RESIDUAL_DOT2: return RES_DOT2;
    case RID_RESIDUAL_FP64: return RES_FP64;
    case RID_RESIDUAL_FP32: return RES_FP32;
    default: return prec == RID_FP64 ? RES_DOT2 : RES_FP64;
  }
}

void residual_batch_setup(const RidBatchJob *bj, int count, rid_dtype dtype, int64_t block_bytes,
                          int ahz_cpw, int acc, void *ws, GroupedHost *out);
hipError_t launch_residual_batch(hipStream_t st, rid_dtype dtype, const void *djobs,
                                 const int4 *dtab, const GroupedHost &gh, int q, int acc,
                                 RidProf *prof);

size_t residual_ws_bytes(int64_t m, int64_t n, int64_t k, int q);
hipError_t launch_residual(hipStream_t st, rid_dtype dtype, int64_t m, int64_t n, int64_t k,
                           const void *A, int64_t lda, const int64_t *J,
                           const double2 *P, int64_t ldp, int q, uint64_t seed,
                           double *sigma, double *hist, void *ws, RidProf *prof, int acc);
