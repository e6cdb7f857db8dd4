// api.hip -- the extern "C" entry points of librid (declared in rid.h):
// argument validation, device selection, workspace, and the order of the
// steps of the randomized ID (Sec. 2), including the redraw on rank(Y) < k.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>

#include "rid_internal.hpp"

// Device scratch of rid_pivqr_static: a file-scope array, one copy on each
// device the library runs on, held until the process ends.  Host code never
// uses the array's name as an address: rid_create looks its device address
// up once per device (scratch_setup) and the entry point passes that.
static __device__ __align__(256) char scratch[RID_STATIC_SCRATCH_BYTES];

namespace {

constexpr int RID_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[RID_MAX_DEVICES];
hipError_t g_scratch_err[RID_MAX_DEVICES];
bool g_scratch_done[RID_MAX_DEVICES];

// With `device` current: the device address of `scratch` on it, looked up
// once per device.
void scratch_setup(int device) {
  if (device < 0 || device >= RID_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
  if (e != hipSuccess) (void)hipGetLastError();
  g_scratch_done[device] = true;
}

// The scratch address of `device` (null if its lookup failed; *err then
// holds the HIP error).
void *scratch_of(int device, hipError_t *err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= RID_MAX_DEVICES || !g_scratch_done[device]) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) {
      err = hipSetDevice(dev);
      changed = (err == hipSuccess);
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

rid_status fail_hip(rid_handle h, hipError_t e) {
  if (h) h->last_hip_error = static_cast<int>(e);
  return RID_ERR_HIP;
}

rid_status ensure_ws(rid_handle h, size_t bytes) {
  const hipError_t e = grow_ws(h, bytes);
  if (e == hipErrorOutOfMemory) {
    h->last_hip_error = static_cast<int>(e);
    return RID_ERR_NOMEM;
  }
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t bytes_sketch(rid_dtype dt, rid_prec pr, int64_t m, int64_t n, int64_t l, bool with_g) {
  WsCarve c(nullptr);
  if (with_g) c.take<double2>(size_t(l) * size_t(m));
  c.take<char>(sketch_ws_bytes(dt, pr, m, n, l));
  return c.off + 256;
}

// Workspace of rid_decompose: Y, perm and gaps persist across the steps; the
// scratch of each step (G + split-K partials, QR, interp, residual) reuses
// one region.
struct DecompWs {
  double2 *Y;
  int64_t *perm;
  double *gaps;
  void *scratch;
  double2 *G;
  void *part;
};

template <class C>
DecompWs carve_decomp(C &c, rid_dtype dt, rid_prec pr, int64_t m, int64_t n, int64_t k,
                      int64_t l) {
  DecompWs d;
  d.Y = c.template take<double2>(size_t(l) * size_t(n));
  d.perm = c.template take<int64_t>(n);
  d.gaps = c.template take<double>(k);
  const size_t base = (c.off + 255) & ~size_t(255);
  c.off = base;
  d.scratch = c.base ? c.base + base : nullptr;
  d.G = c.template take<double2>(size_t(l) * size_t(m));
  d.part = c.template take<char>(sketch_ws_bytes(dt, pr, m, n, l));
  return d;
}

size_t bytes_decomp(rid_dtype dt, rid_prec pr, int64_t m, int64_t n, int64_t k, int64_t l,
                    int q, int qr_kind, int sketch_kind = RID_SKETCH_GAUSSIAN) {
  WsCarve c(nullptr);
  carve_decomp(c, dt, pr, m, n, k, l);
  // the region after `scratch` must also hold each later step's workspace
  WsCarve c2(nullptr);
  c2.take<double2>(size_t(l) * size_t(n));
  c2.take<int64_t>(n);
  c2.take<double>(k);
  const size_t base = (c2.off + 255) & ~size_t(255);
  size_t need = c.off;
  const size_t srft = (sketch_kind == RID_SKETCH_SRFT && srft_fft_ok(pr, m, l))
                          ? srft_sketch_ws_bytes(m, n, l)
                          : 0;
  const size_t others[] = {pivqr_ws_bytes(l, n, k, qr_kind), interp_ws_bytes(n, k),
                           residual_ws_bytes(m, n, k, q), srft};
  for (size_t o : others)
    if (base + o > need) need = base + o;
  return need + 256;
}

}  // namespace

thread_local bool rid_tl_short_blocks = false;

size_t ws_grow_bytes(const rid_ctx *h, size_t bytes) {
  if (bytes <= h->ws_bytes) return 0;
  const size_t exact = (bytes + 4095) & ~size_t(4095);
  const size_t want = h->ws_bytes + h->ws_bytes / 2;
  return (want < exact) ? exact : ((want + 4095) & ~size_t(4095));
}

size_t ws_held_bytes(const rid_ctx *h) { return h->ws_bytes + h->retired_bytes; }

void release_ws(rid_handle h) {
  DeviceGuard g(h->device);
  if (h->ws) (void)hipFree(h->ws);
  for (void *p : h->retired) (void)hipFree(p);
  h->ws = nullptr;
  h->ws_bytes = 0;
  h->retired.clear();
  h->retired_bytes = 0;
}

hipError_t grow_ws(rid_handle h, size_t bytes) {
  if (bytes <= h->ws_bytes) return hipSuccess;
  const size_t exact = (bytes + 4095) & ~size_t(4095);
  size_t want = ws_grow_bytes(h, bytes);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess && want > exact) {
    (void)hipGetLastError();
    e = hipMalloc(&p, exact);
    want = exact;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  if (h->ws) {
    h->retired.push_back(h->ws);
    h->retired_bytes += h->ws_bytes;
  }
  h->ws = p;
  h->ws_bytes = want;
  return hipSuccess;
}

size_t decomp_ws_bytes(rid_dtype dt, rid_prec pr, int64_t m, int64_t n, int64_t k, int64_t l,
                       int q) {
  return std::max(bytes_decomp(dt, pr, m, n, k, l, q, RID_QR_HOUSEHOLDER),
                  bytes_decomp(dt, pr, m, n, k, l, q, RID_QR_CGS2));
}

extern "C" {

const char *rid_status_string(int status) {
  switch (status) {
    case RID_OK: return "RID_OK";
    case RID_ERR_INVALID_ARG: return "RID_ERR_INVALID_ARG";
    case RID_ERR_UNSUPPORTED: return "RID_ERR_UNSUPPORTED";
    case RID_ERR_NOMEM: return "RID_ERR_NOMEM";
    case RID_ERR_HIP: return "RID_ERR_HIP";
    case RID_ERR_RANK: return "RID_ERR_RANK";
    default: return "RID_ERR_UNKNOWN";
  }
}

rid_status rid_create(rid_handle *h, int device) {
  if (!h) return RID_ERR_INVALID_ARG;
  *h = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return RID_ERR_HIP;
  if (device < 0 || device >= count) return RID_ERR_INVALID_ARG;
  rid_ctx *c = new (std::nothrow) rid_ctx();
  if (!c) return RID_ERR_NOMEM;
  c->device = device;
  DeviceGuard g(device);
  if (g.err != hipSuccess) {
    delete c;
    return RID_ERR_HIP;
  }
  e = hipMalloc(&c->d_status, 256);
  if (e != hipSuccess) {
    delete c;
    return RID_ERR_NOMEM;
  }
  e = hipMemset(c->d_status, 0, 256);
  if (e != hipSuccess) {
    (void)hipFree(c->d_status);
    delete c;
    return RID_ERR_HIP;
  }
  scratch_setup(device);
  *h = c;
  return RID_OK;
}

rid_status rid_destroy(rid_handle h) {
  if (!h) return RID_OK;
  DeviceGuard g(h->device);
  for (hipEvent_t e : h->prof.pool) (void)hipEventDestroy(e);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->ws) (void)hipFree(h->ws);
  for (void *p : h->retired) (void)hipFree(p);
  if (h->d_status) (void)hipFree(h->d_status);
  delete h;
  return RID_OK;
}

int rid_last_hip_error(rid_handle h) { return h ? h->last_hip_error : 0; }

rid_status rid_reserve(rid_handle h, int64_t max_m, int64_t max_n, int64_t max_l,
                       int64_t max_k) {
  if (!h || max_m < 0 || max_n < 0 || max_l < 0 || max_k < 0) return RID_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  size_t need = 0;
  for (rid_prec pr : {RID_FP64, RID_FP32, RID_BF16X3}) {
    const size_t sk = bytes_sketch(RID_C128, pr, max_m, max_n, max_l, true);
    const size_t d = std::max(bytes_decomp(RID_C128, pr, max_m, max_n, max_k, max_l, 1,
                                           RID_QR_HOUSEHOLDER, h->sketch_kind),
                              bytes_decomp(RID_C128, pr, max_m, max_n, max_k, max_l, 1,
                                           RID_QR_CGS2, h->sketch_kind));
    if (sk > need) need = sk;
    if (d > need) need = d;
  }
  return ensure_ws(h, need);
}

rid_status rid_gaussian(rid_handle h, hipStream_t stream, int64_t rows, int64_t cols,
                        uint64_t seed, uint32_t stream_id, void *out, int64_t ld) {
  if (!h || rows < 0 || cols < 0 || rows > 0xFFFFFFFFll || ld < cols || (rows * cols > 0 && !out))
    return RID_ERR_INVALID_ARG;
  if (out && !aligned(out, 16)) return RID_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  hipError_t e = launch_gaussian(stream, rows, cols, seed, stream_id, static_cast<double2 *>(out), ld);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_set_sketch(rid_handle h, int kind) {
  if (!h || (kind != RID_SKETCH_GAUSSIAN && kind != RID_SKETCH_SRFT)) return RID_ERR_INVALID_ARG;
  h->sketch_kind = kind;
  return RID_OK;
}

rid_status rid_srft_operator(rid_handle h, hipStream_t stream, int64_t rows, int64_t m,
                             uint64_t seed, void *out, int64_t ld) {
  if (!h || rows < 0 || m < 1 || m > 0x7FFFFFFFll || ld < m || (rows > 0 && !out))
    return RID_ERR_INVALID_ARG;
  if (out && !aligned(out, 16)) return RID_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  hipError_t e = launch_srft(stream, rows, m, seed, static_cast<double2 *>(out), ld);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

static rid_status check_sketch_args(rid_handle h, rid_dtype dtype, rid_prec prec, int64_t m,
                                    int64_t n, int64_t l, const void *A, int64_t lda, void *Y,
                                    int64_t ldy) {
  if (!h || m < 0 || n < 0 || l < 1 || l > 0xFFFFFFFFll) return RID_ERR_INVALID_ARG;
  if (lda < (m > 1 ? m : 1) || ldy < l) return RID_ERR_INVALID_ARG;
  if (n > 0 && (!Y || !aligned(Y, 16))) return RID_ERR_INVALID_ARG;
  if (m > 0 && n > 0 && !A) return RID_ERR_INVALID_ARG;
  if (dtype != RID_C128 && dtype != RID_C64) return RID_ERR_INVALID_ARG;
  if (!prec_valid(prec)) return RID_ERR_INVALID_ARG;
  if (A && !aligned(A, dtype == RID_C128 ? 16 : 8)) return RID_ERR_INVALID_ARG;
  if (!sketch_supported(dtype, prec)) return RID_ERR_UNSUPPORTED;
  if (h->sketch_kind == RID_SKETCH_SRFT && m > 0x7FFFFFFFll) return RID_ERR_UNSUPPORTED;
  return RID_OK;
}

static rid_status zero_fill(rid_handle h, hipStream_t stream, void *Y, int64_t ldy, int64_t l,
                            int64_t n) {
  // Y = 0 when m == 0 (an empty sum)
  hipError_t e = launch_zero(stream, l, n, static_cast<double2 *>(Y), ldy);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_sketch_explicit(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                               int64_t m, int64_t n, int64_t l, const void *A, int64_t lda,
                               const void *G, int64_t ldg, void *Y, int64_t ldy) {
  rid_status s = check_sketch_args(h, dtype, prec, m, n, l, A, lda, Y, ldy);
  if (s != RID_OK) return s;
  if (ldg < (m > 1 ? m : 1) || (m > 0 && (!G || !aligned(G, 16)))) return RID_ERR_INVALID_ARG;
  if (n == 0) return RID_OK;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  if (m == 0) return zero_fill(h, stream, Y, ldy, l, n);
  s = ensure_ws(h, bytes_sketch(dtype, prec, m, n, l, false));
  if (s != RID_OK) return s;
  WsCarve c(h->ws);
  void *part = c.take<char>(sketch_ws_bytes(dtype, prec, m, n, l));
  hipError_t e = launch_sketch(stream, dtype, prec, m, n, l, A, lda,
                               static_cast<const double2 *>(G), ldg, static_cast<double2 *>(Y),
                               ldy, part, &h->prof);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_sketch(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                      int64_t m, int64_t n, int64_t l, const void *A, int64_t lda,
                      uint64_t seed, void *Y, int64_t ldy) {
  rid_status s = check_sketch_args(h, dtype, prec, m, n, l, A, lda, Y, ldy);
  if (s != RID_OK) return s;
  if (n == 0) return RID_OK;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  if (m == 0) return zero_fill(h, stream, Y, ldy, l, n);
  if (h->sketch_kind == RID_SKETCH_SRFT && srft_fft_ok(prec, m, l)) {
    s = ensure_ws(h, srft_sketch_ws_bytes(m, n, l));
    if (s != RID_OK) return s;
    const hipError_t e = launch_srft_sketch(stream, dtype, m, n, l, A, lda, seed,
                                            static_cast<double2 *>(Y), ldy, h->ws, &h->prof);
    return e == hipSuccess ? RID_OK : fail_hip(h, e);
  }
  s = ensure_ws(h, bytes_sketch(dtype, prec, m, n, l, true));
  if (s != RID_OK) return s;
  WsCarve c(h->ws);
  double2 *G = c.take<double2>(size_t(l) * size_t(m));
  void *part = c.take<char>(sketch_ws_bytes(dtype, prec, m, n, l));
  hipError_t e = launch_operator(stream, h->sketch_kind, l, m, seed, G, m);
  if (e != hipSuccess) return fail_hip(h, e);
  e = launch_sketch(stream, dtype, prec, m, n, l, A, lda, G, m, static_cast<double2 *>(Y), ldy,
                    part, &h->prof);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_pivqr(rid_handle h, hipStream_t stream, int64_t l, int64_t n, int64_t k,
                     void *Y, int64_t ldy, int64_t *perm, double *gaps, double rank_tol) {
  if (!h || k < 1 || k > l || k > n || ldy < l || !Y || !perm || !aligned(Y, 16) ||
      !(rank_tol >= 0.0) || !std::isfinite(rank_tol) || n > 0x7FFFFFFFll)
    return RID_ERR_INVALID_ARG;
  if (!pivqr_supported(l)) return RID_ERR_UNSUPPORTED;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  if (h->qr_kind == RID_QR_CGS2 && k > 1024) return RID_ERR_UNSUPPORTED;
  rid_status s = ensure_ws(h, pivqr_ws_bytes(l, n, k, h->qr_kind));
  if (s != RID_OK) return s;
  hipError_t e = launch_pivqr(stream, l, n, k, static_cast<double2 *>(Y), ldy, perm, gaps,
                              rank_tol, h->ws, h->d_status, &h->prof, h->qr_kind);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_pivqr_static(rid_handle h, hipStream_t stream, int64_t l, int64_t n, int64_t k,
                            void *Y, int64_t ldy, int64_t *perm, double *gaps,
                            double rank_tol) {
  if (!h || k < 1 || k > l || k > n || ldy < l || !Y || !perm || !aligned(Y, 16) ||
      !(rank_tol >= 0.0) || !std::isfinite(rank_tol) || n > 0x7FFFFFFFll)
    return RID_ERR_INVALID_ARG;
  if (!pivqr_supported(l)) return RID_ERR_UNSUPPORTED;
  if (h->qr_kind == RID_QR_CGS2 && k > 1024) return RID_ERR_UNSUPPORTED;
  if (pivqr_ws_bytes(l, n, k, h->qr_kind) > size_t(RID_STATIC_SCRATCH_BYTES))
    return RID_ERR_NOMEM;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  hipError_t e = hipSuccess;
  void *ws = scratch_of(h->device, &e);
  if (!ws) return fail_hip(h, e);
  e = launch_pivqr(stream, l, n, k, static_cast<double2 *>(Y), ldy, perm, gaps, rank_tol, ws,
                   h->d_status, nullptr, h->qr_kind);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_interp(rid_handle h, hipStream_t stream, int64_t n, int64_t k, const void *R,
                      int64_t ldr, const int64_t *J, void *P, int64_t ldp) {
  if (!h || k < 1 || k > n || ldr < k || ldp < k || !R || !J || !P || !aligned(R, 16) ||
      !aligned(P, 16) || n > 0x7FFFFFFFll)
    return RID_ERR_INVALID_ARG;
  if (!interp_supported(k)) return RID_ERR_UNSUPPORTED;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  rid_status s = ensure_ws(h, interp_ws_bytes(n, k));
  if (s != RID_OK) return s;
  hipError_t e = launch_interp(stream, n, k, static_cast<const double2 *>(R), ldr, J,
                               static_cast<double2 *>(P), ldp, h->ws, &h->prof);
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_residual(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                        int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                        const int64_t *J, const void *P, int64_t ldp, int q, uint64_t seed,
                        double *sigma, double *hist) {
  if (!h || m < 1 || n < 1 || k < 0 || k > n || q < 1 || lda < m || !A || !sigma ||
      (k > 0 && (!J || !P || ldp < k)) || (P && !aligned(P, 16)))
    return RID_ERR_INVALID_ARG;
  if (dtype != RID_C128 && dtype != RID_C64) return RID_ERR_INVALID_ARG;
  if (!prec_valid(prec)) return RID_ERR_INVALID_ARG;
  if (!aligned(A, dtype == RID_C128 ? 16 : 8)) return RID_ERR_INVALID_ARG;
  if (k > 1024) return RID_ERR_UNSUPPORTED;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  rid_status s = ensure_ws(h, residual_ws_bytes(m, n, k, q));
  if (s != RID_OK) return s;
  hipError_t e = launch_residual(stream, dtype, m, n, k, A, lda, J,
                                 static_cast<const double2 *>(P), k > 0 ? ldp : 1, q, seed,
                                 sigma, hist, h->ws, &h->prof, res_acc(h->residual_kind, prec));
  return e == hipSuccess ? RID_OK : fail_hip(h, e);
}

rid_status rid_set_residual(rid_handle h, int kind) {
  if (!h || kind < RID_RESIDUAL_AUTO || kind > RID_RESIDUAL_FP32) return RID_ERR_INVALID_ARG;
  h->residual_kind = kind;
  return RID_OK;
}

rid_status rid_set_qr(rid_handle h, int kind) {
  if (!h || (kind != RID_QR_HOUSEHOLDER && kind != RID_QR_CGS2)) return RID_ERR_INVALID_ARG;
  h->qr_kind = kind;
  return RID_OK;
}

rid_status rid_profile(rid_handle h, int enable) {
  if (!h) return RID_ERR_INVALID_ARG;
  if (enable) {
    h->prof.used = 0;
    h->prof.recs.clear();
  }
  h->prof.on = enable != 0;
  return RID_OK;
}

rid_status rid_profile_read(rid_handle h, int kernel, double *total_ms, int64_t *launches) {
  if (!h || kernel < 0 || kernel >= RID_KERNEL_COUNT) return RID_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  double tot = 0.0;
  int64_t cnt = 0;
  for (const auto &r : h->prof.recs) {
    if (r.first != kernel) continue;
    hipEvent_t a = h->prof.pool[r.second], b = h->prof.pool[r.second + 1];
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) return fail_hip(h, e);
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return RID_OK;
}

rid_status rid_query_status(rid_handle h, hipStream_t stream) {
  if (!h) return RID_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  int v = 0;
  hipError_t e = hipMemcpyAsync(&v, h->d_status, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail_hip(h, e);
  return static_cast<rid_status>(v);
}

}  // extern "C"

namespace {

// The whole ID (Sec. 2).  Draw a = 0, 1, ... uses the operator of seed + a,
// except that a caller-supplied G0 (l x m, row-major, ldg) replaces the
// first draw's operator.
rid_status decompose_impl(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                          int64_t m, int64_t n, int64_t k, int64_t l, const void *A,
                          int64_t lda, const double2 *G0, int64_t ldg, uint64_t seed, int q,
                          int max_retries, double rank_tol, int64_t *J, void *P, int64_t ldp,
                          double *sigma, uint64_t *seed_used) {
  if (!h || k < 1 || k > l || k > n || l > m || q < 1 || max_retries < 0 || lda < m || !A ||
      !J || !P || !sigma || ldp < k || !aligned(P, 16) || !(rank_tol >= 0.0) ||
      !std::isfinite(rank_tol) || n > 0x7FFFFFFFll || l > 0xFFFFFFFFll)
    return RID_ERR_INVALID_ARG;
  if (dtype != RID_C128 && dtype != RID_C64) return RID_ERR_INVALID_ARG;
  if (!prec_valid(prec)) return RID_ERR_INVALID_ARG;
  if (!aligned(A, dtype == RID_C128 ? 16 : 8)) return RID_ERR_INVALID_ARG;
  if (G0 && (ldg < m || !aligned(G0, 16))) return RID_ERR_INVALID_ARG;
  if (!sketch_supported(dtype, prec)) return RID_ERR_UNSUPPORTED;
  if (!pivqr_supported(l) || !interp_supported(k)) return RID_ERR_UNSUPPORTED;
  if (h->sketch_kind == RID_SKETCH_SRFT && m > 0x7FFFFFFFll) return RID_ERR_UNSUPPORTED;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  if (h->qr_kind == RID_QR_CGS2 && k > 1024) return RID_ERR_UNSUPPORTED;
  const bool fft = h->sketch_kind == RID_SKETCH_SRFT && srft_fft_ok(prec, m, l);
  rid_status s =
      ensure_ws(h, bytes_decomp(dtype, prec, m, n, k, l, q, h->qr_kind, h->sketch_kind));
  if (s != RID_OK) return s;
  WsCarve c(h->ws);
  const DecompWs d = carve_decomp(c, dtype, prec, m, n, k, l);
  for (int attempt = 0; attempt <= max_retries; ++attempt) {
    const uint64_t sd = seed + static_cast<uint64_t>(attempt);
    hipError_t e;
    if (G0 && attempt == 0) {
      e = launch_sketch(stream, dtype, prec, m, n, l, A, lda, G0, ldg, d.Y, l, d.part,
                        &h->prof);
    } else if (fft) {
      e = launch_srft_sketch(stream, dtype, m, n, l, A, lda, sd, d.Y, l, d.scratch, &h->prof);
    } else {
      e = launch_operator(stream, h->sketch_kind, l, m, sd, d.G, m);
      if (e == hipSuccess)
        e = launch_sketch(stream, dtype, prec, m, n, l, A, lda, d.G, m, d.Y, l, d.part,
                          &h->prof);
    }
    if (e == hipSuccess)
      e = launch_pivqr(stream, l, n, k, d.Y, l, d.perm, d.gaps, rank_tol, d.scratch,
                       h->d_status, &h->prof, h->qr_kind);
    if (e != hipSuccess) return fail_hip(h, e);
    int st = 0;
    e = hipMemcpyAsync(&st, h->d_status, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail_hip(h, e);
    if (st == RID_ERR_RANK) continue;
    if (st != RID_OK) return RID_ERR_HIP;
    e = hipMemcpyAsync(J, d.perm, size_t(k) * sizeof(int64_t), hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
      e = launch_interp(stream, n, k, d.Y, l, d.perm, static_cast<double2 *>(P), ldp,
                        d.scratch, &h->prof);
    if (e == hipSuccess)
      e = launch_residual(stream, dtype, m, n, k, A, lda, d.perm,
                          static_cast<const double2 *>(P), ldp, q, sd, sigma, nullptr, d.scratch,
                          &h->prof, res_acc(h->residual_kind, prec));
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail_hip(h, e);
    if (seed_used) *seed_used = sd;
    return RID_OK;
  }
  return RID_ERR_RANK;
}

}  // namespace

extern "C" {

rid_status rid_decompose(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                         int64_t m, int64_t n, int64_t k, int64_t l, const void *A,
                         int64_t lda, uint64_t seed, int q, int max_retries, double rank_tol,
                         int64_t *J, void *P, int64_t ldp, double *sigma,
                         uint64_t *seed_used) {
  return decompose_impl(h, stream, dtype, prec, m, n, k, l, A, lda, nullptr, 0, seed, q,
                        max_retries, rank_tol, J, P, ldp, sigma, seed_used);
}

rid_status rid_decompose_explicit(rid_handle h, hipStream_t stream, rid_dtype dtype,
                                  rid_prec prec, int64_t m, int64_t n, int64_t k, int64_t l,
                                  const void *A, int64_t lda, const void *G0, int64_t ldg,
                                  uint64_t seed, int q, int max_retries, double rank_tol,
                                  int64_t *J, void *P, int64_t ldp, double *sigma,
                                  uint64_t *seed_used) {
  if (!G0) return RID_ERR_INVALID_ARG;
  return decompose_impl(h, stream, dtype, prec, m, n, k, l, A, lda,
                        static_cast<const double2 *>(G0), ldg, seed, q, max_retries, rank_tol, J,
                        P, ldp, sigma, seed_used);
}

rid_status rid_svd(rid_handle h, hipStream_t stream, rid_dtype dtype, int64_t m, int64_t n,
                   int64_t k, const void *A, int64_t lda, const int64_t *J, const void *P,
                   int64_t ldp, void *U, int64_t ldu, double *S, void *V, int64_t ldv,
                   int *sweeps) {
  if (!h || k < 1 || k > m || k > n || lda < m || ldp < k || ldu < m || ldv < n || !A || !J ||
      !P || !U || !S || !V || !aligned(P, 16) || !aligned(U, 16) || !aligned(V, 16) ||
      m > (int64_t(1) << 22) || n > 0x7FFFFFFFll)
    return RID_ERR_INVALID_ARG;
  if (dtype != RID_C128 && dtype != RID_C64) return RID_ERR_INVALID_ARG;
  if (!aligned(A, dtype == RID_C128 ? 16 : 8)) return RID_ERR_INVALID_ARG;
  if (!svd_supported(k)) return RID_ERR_UNSUPPORTED;
  DeviceGuard g(h->device);
  if (g.err != hipSuccess) return fail_hip(h, g.err);
  rid_status s = ensure_ws(h, svd_ws_bytes(m, n, k));
  if (s != RID_OK) return s;
  int bad = 0, used = 0;
  const hipError_t e = launch_svd(stream, dtype, m, n, k, A, lda, J,
                                  static_cast<const double2 *>(P), ldp, static_cast<double2 *>(U),
                                  ldu, S, static_cast<double2 *>(V), ldv, h->ws, &bad, &used);
  if (e == hipSuccess) {
    const hipError_t e2 = hipStreamSynchronize(stream);
    if (e2 != hipSuccess) return fail_hip(h, e2);
  }
  if (e != hipSuccess) return fail_hip(h, e);
  if (sweeps) *sweeps = used;
  return bad ? RID_ERR_RANK : RID_OK;
}

}  // extern "C"
