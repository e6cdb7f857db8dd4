// batched.hip -- many independent IDs of uneven sizes in one call
// (rid_decompose_batched).  Every step of the ID runs as one launch over all
// jobs: blocks find their (job, block) pair in host-built tables, so a batch
// costs the same number of launches as one ID.  The launch sequence is
// captured into a HIP graph and replayed on the caller's stream.
//
// The pivoted QR takes one grouped launch per step: every job's sketch is
// split into 64-column workgroups as in the single-ID QR, and a job whose
// k steps are done leaves the later launches at once.  A job whose sketch
// has rank < k is redrawn with seed + 1 (Sec. 2), up to max_retries times,
// in a follow-up batch of the failures.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "rid_internal.hpp"

namespace {

struct OpJob {
  int64_t rows, cols, ld;
  uint64_t seed;
  double2 *out;
  int kind;
};

// ---------------------------------------------------------------- operators
__global__ __launch_bounds__(256) void operator_grouped_kernel(const OpJob *__restrict__ jobs,
                                                               const int4 *__restrict__ tab) {
  const int4 en = tab[blockIdx.x];
  const OpJob &jb = jobs[en.x];
  const int64_t total = jb.rows * jb.cols;
  for (int64_t e = int64_t(en.y) * 256 + threadIdx.x; e < total; e += int64_t(en.z) * 256) {
    const int64_t i = e / jb.cols;
    const int64_t p = e - i * jb.cols;
    double2 g;
    if (jb.kind == RID_SKETCH_SRFT) {
      uint32_t c[4] = {static_cast<uint32_t>(i), static_cast<uint32_t>(uint64_t(i) >> 32), 0u, 6u};
      rid_philox10(c, static_cast<uint32_t>(jb.seed), static_cast<uint32_t>(jb.seed >> 32));
      int64_t si = static_cast<int64_t>(floor(rid_u52(c[0], c[1]) * static_cast<double>(jb.cols)));
      if (si >= jb.cols) si = jb.cols - 1;
      uint32_t d[4] = {static_cast<uint32_t>(p), static_cast<uint32_t>(uint64_t(p) >> 32), 0u, 5u};
      rid_philox10(d, static_cast<uint32_t>(jb.seed), static_cast<uint32_t>(jb.seed >> 32));
      const int64_t r = static_cast<int64_t>((static_cast<uint64_t>(si) * static_cast<uint64_t>(p)) %
                                             static_cast<uint64_t>(jb.cols));
      const double ang = 6.283185307179586476925286766559 *
                         (rid_u52(d[0], d[1]) - static_cast<double>(r) / static_cast<double>(jb.cols));
      g = make_double2(cos(ang), sin(ang));
    } else {
      g = rid_gauss(jb.seed, 0u, static_cast<uint32_t>(i), static_cast<uint64_t>(p));
    }
    jb.out[i * jb.ld + p] = g;
  }
}

// ---------------------------------------------------------------- host side
struct Buf {
  std::vector<char> bytes;
  template <class T>
  size_t put(const T *p, size_t count) {
    size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + sizeof(T) * count);
    if (count) memcpy(bytes.data() + off, p, sizeof(T) * count);
    return off;
  }
};

bool use_graph() {
  const char *e = getenv("RID_BATCH_GRAPH");
  return !(e && e[0] == '0');
}

// The QR of a batch: one launch per pivot step over all jobs, two columns
// in flight per wave (5.1-5.3 ms per 512-job batch; RID_BATCH_QR=1 or 4,
// one or four at a time, took 5.4 and 5.3 ms).  RID_BATCH_QR=jobs selects
// one launch with a workgroup per job for all its steps instead (12.9 ms:
// a big job's steps run one after another on one CU).  The arithmetic is
// the same: J and R agree bit for bit.
int qr_mode() {
  const char *e = getenv("RID_BATCH_QR");
  if (e && e[0] == 'j') return 0;
  if (e && (e[0] == '1' || e[0] == '4')) return e[0] - '0';  // columns in flight per wave
  return 2;
}

}  // namespace

// The grouped sketch is built for FP64 and FP32 products.
bool batch_prec_supported(rid_prec prec) {
  return prec == RID_FP64 || prec == RID_FP32 || prec == RID_BF16X2 || prec == RID_BF16X3;
}

bool batch_job_supported(const RidBatchJob &j) {
  return j.l <= 256 && j.k <= 256 && sketch_pick_mt(j.l) > 0;
}

// Runs one batch (each job once, with the seeds in bj); writes per-job
// status (host).  With need_only non-null it only plans: the workspace size
// goes there and nothing touches the device.
static hipError_t run_batch_impl(rid_handle h, hipStream_t stream, rid_dtype dtype,
                                 rid_prec prec, const RidBatchJob *bj, int count, int q,
                                 double rank_tol, int *status, RidProf *prof, size_t *need_only) {
  // ---- plans and workspace layout
  std::vector<SketchJob> sk(count);
  std::vector<OpJob> op(count);
  std::vector<PivJob> qr(count);
  std::vector<InterpJob> in(count);
  std::vector<int> mt(count);
  int kmax = 1;
  for (int i = 0; i < count; ++i) kmax = std::max<int>(kmax, static_cast<int>(bj[i].k));
  // persistent region: Y, mark, status; scratch region: G + partials, or the
  // residual workspace (the sketch is done before the residual starts)
  WsCarve pc(nullptr);
  std::vector<size_t> offY(count), offMark(count);
  for (int i = 0; i < count; ++i) {
    offY[i] = pc.take_off<double2>(size_t(bj[i].l) * size_t(bj[i].n));
    offMark[i] = pc.take_off<int>(bj[i].n);
  }
  const size_t offStatus = pc.take_off<int>(count);
  const size_t persist = (pc.off + 255) & ~size_t(255);
  WsCarve sc(nullptr);
  std::vector<size_t> offG(count), offPart(count), offPl(count);
  const int64_t pchunk = h->batch_sketch_rows;
  const bool bf16 = prec == RID_BF16X2 || prec == RID_BF16X3;
  const int nterms = prec == RID_BF16X2 ? 2 : 3;
  for (int i = 0; i < count; ++i) {
    mt[i] = sketch_pick_mt(bj[i].l);
    // the reduced-precision kernels cover (mt + 1) / 2 row tiles of Y, so
    // tile counts 2c - 1 and 2c share one launch
    if (prec != RID_FP64) mt[i] = (mt[i] + 1) / 2 * 2;
    const int64_t S = (bj[i].m + pchunk - 1) / pchunk;
    offG[i] = sc.take_off<double2>(size_t(bj[i].l) * size_t(bj[i].m));
    const size_t el = prec == RID_FP64 ? sizeof(double) : sizeof(float);
    offPart[i] = sc.take_off<char>(size_t(S) * size_t(2 * bj[i].l) * size_t(bj[i].n) * el);
    // bf16 planes: 16 rows per row tile of the bucket, K padded to 16
    if (bf16)
      offPl[i] = sc.take_off<uint16_t>(size_t(nterms) * size_t(8 * mt[i]) *
                                       size_t(2 * ((bj[i].m + 15) / 16 * 16)));
  }
  // the QR workspace reuses the scratch region too (G is dead by then)
  WsCarve qc(nullptr);
  std::vector<size_t> offQr(count);
  for (int i = 0; i < count; ++i)
    offQr[i] = qc.take_off<char>(pivqr_job_ws_bytes(bj[i].l, bj[i].n));
  GroupedHost res;
  const int acc = res_acc(h->residual_kind, prec);
  residual_batch_setup(bj, count, dtype, h->batch_res_block_bytes, h->batch_ahz_cpw, acc, nullptr,
                       &res);
  const size_t scratch = std::max(std::max(sc.off, qc.off), res.ws_bytes) + 256;

  // ---- descriptor + table upload region goes first
  // (sizes are known only after the tables are built; build them with a
  // provisional base, then fix pointers once the base is known)
  Buf tabs;
  std::vector<int4> t_op, t_red, t_qr, t_in;
  std::vector<std::vector<int4>> t_sk;
  std::vector<int> mts;
  for (int i = 0; i < count; ++i) {
    const int64_t tot = bj[i].l * bj[i].m;
    const int nb = static_cast<int>(std::min<int64_t>((tot + 255) / 256, 256));
    for (int b = 0; b < nb; ++b) t_op.push_back(make_int4(i, b, nb, 0));
    const int64_t totY = 2 * bj[i].l * bj[i].n;
    const int nr = static_cast<int>(std::min<int64_t>((totY + 255) / 256, 64));
    for (int b = 0; b < nr; ++b) t_red.push_back(make_int4(i, b, nr, 0));
    int bucket = -1;
    for (size_t u = 0; u < mts.size(); ++u)
      if (mts[u] == mt[i]) bucket = static_cast<int>(u);
    if (bucket < 0) {
      mts.push_back(mt[i]);
      t_sk.emplace_back();
      bucket = static_cast<int>(mts.size()) - 1;
    }
    const int64_t cols = sketch_batch_cols(prec);
    const int64_t nbx = (bj[i].n + cols - 1) / cols;
    const int64_t S = (bj[i].m + pchunk - 1) / pchunk;
    for (int64_t s = 0; s < S; ++s)
      for (int64_t x = 0; x < nbx; ++x)
        t_sk[bucket].push_back(make_int4(i, static_cast<int>(x), static_cast<int>(s), 0));
    const int64_t nq = interp_blocks(bj[i].n);
    for (int64_t x = 0; x < nq; ++x) t_in.push_back(make_int4(i, static_cast<int>(x), 0, 0));
  }
  // the QR table by k, largest first: the launch of step t covers only the
  // prefix of jobs that still have step t (k >= t), and picks its rows per
  // lane from their largest l
  std::vector<int> by_k(count);
  std::iota(by_k.begin(), by_k.end(), 0);
  std::stable_sort(by_k.begin(), by_k.end(), [&](int a, int b) { return bj[a].k > bj[b].k; });
  std::vector<int64_t> qr_live(kmax + 1, 0), qr_lmax(kmax + 1, 1);
  for (int i : by_k) {
    const int64_t nbq = pivqr_blocks(bj[i].n);
    for (int64_t x = 0; x < nbq; ++x)
      t_qr.push_back(make_int4(i, static_cast<int>(x), static_cast<int>(nbq), 0));
    for (int64_t t = 0; t <= bj[i].k && t <= kmax; ++t) {
      qr_live[t] = static_cast<int64_t>(t_qr.size());
      qr_lmax[t] = std::max<int64_t>(qr_lmax[t], bj[i].l);
    }
  }

  // the per-job QR launch takes the largest jobs first
  std::vector<int> qr_order(count);
  std::iota(qr_order.begin(), qr_order.end(), 0);
  std::stable_sort(qr_order.begin(), qr_order.end(), [&](int a, int b) {
    return double(bj[a].k + 1) * double(bj[a].n) * double(bj[a].l) >
           double(bj[b].k + 1) * double(bj[b].n) * double(bj[b].l);
  });

  // descriptor region size
  const size_t nbuck = mts.size();
  size_t tabbytes;
  {
    Buf probe;
    probe.put(sk.data(), count);
    probe.put(op.data(), count);
    probe.put(qr.data(), count);
    probe.put(in.data(), count);
    probe.put(res.jobs.data(), res.jobs.size());
    probe.put(t_op.data(), t_op.size());
    probe.put(t_red.data(), t_red.size());
    probe.put(t_qr.data(), t_qr.size());
    probe.put(t_in.data(), t_in.size());
    probe.put(res.tab.data(), res.tab.size());
    probe.put(qr_order.data(), qr_order.size());
    for (size_t u = 0; u < nbuck; ++u) probe.put(t_sk[u].data(), t_sk[u].size());
    tabbytes = (probe.bytes.size() + 255) & ~size_t(255);
  }
  const size_t total = tabbytes + persist + scratch + 256;
  if (need_only) {
    *need_only = total;
    return hipSuccess;
  }
  // the residual descriptors need the final scratch base: set it up now
  hipError_t err = hipSuccess;
  {
    const hipError_t e = grow_ws(h, total);
    if (e != hipSuccess) return e;
  }
  char *base = static_cast<char *>(h->ws);
  char *pbase = base + tabbytes;
  char *sbase = pbase + persist;
  residual_batch_setup(bj, count, dtype, h->batch_res_block_bytes, h->batch_ahz_cpw, acc, sbase,
                       &res);
  int *dstatus = reinterpret_cast<int *>(pbase + offStatus);
  for (int i = 0; i < count; ++i) {
    double2 *Y = reinterpret_cast<double2 *>(pbase + offY[i]);
    int *mark = reinterpret_cast<int *>(pbase + offMark[i]);
    double2 *G = reinterpret_cast<double2 *>(sbase + offG[i]);
    sk[i] = SketchJob{bj[i].m, bj[i].n, bj[i].l, bj[i].lda, bj[i].m, pchunk, bj[i].A, G,
                      sbase + offPart[i], Y, (bj[i].m + pchunk - 1) / pchunk, 0,
                      nullptr, 0, 0, 0};
    if (bf16) {
      sk[i].planes = sbase + offPl[i];
      sk[i].prow = 8 * mt[i];
      sk[i].ldk = 2 * ((bj[i].m + 15) / 16 * 16);
      sk[i].pstride = sk[i].prow * sk[i].ldk;
    }
    op[i] = OpJob{bj[i].l, bj[i].m, bj[i].m, bj[i].seed, G, h->sketch_kind};
    qr[i] = PivJob{bj[i].l, bj[i].n, bj[i].k, bj[i].l, Y, bj[i].J, mark, dstatus + i, rank_tol,
                   nullptr, nullptr, nullptr, nullptr, nullptr};
    pivqr_job_carve(sbase + offQr[i], qr[i]);
    in[i] = InterpJob{bj[i].n, bj[i].k, bj[i].l, bj[i].ldp, Y, bj[i].J, bj[i].P, mark};
  }
  const size_t o_sk = tabs.put(sk.data(), count);
  const size_t o_op = tabs.put(op.data(), count);
  const size_t o_qr = tabs.put(qr.data(), count);
  const size_t o_in = tabs.put(in.data(), count);
  const size_t o_res = tabs.put(res.jobs.data(), res.jobs.size());
  const size_t o_top = tabs.put(t_op.data(), t_op.size());
  const size_t o_tred = tabs.put(t_red.data(), t_red.size());
  const size_t o_tqr = tabs.put(t_qr.data(), t_qr.size());
  const size_t o_tin = tabs.put(t_in.data(), t_in.size());
  const size_t o_tres = tabs.put(res.tab.data(), res.tab.size());
  const size_t o_qord = tabs.put(qr_order.data(), qr_order.size());
  std::vector<int64_t> skoff(nbuck), skcnt(nbuck);
  size_t o_tsk0 = 0;
  for (size_t u = 0; u < nbuck; ++u) {
    const size_t o = tabs.put(t_sk[u].data(), t_sk[u].size());
    if (u == 0) o_tsk0 = o;
    skoff[u] = static_cast<int64_t>((o - o_tsk0) / sizeof(int4));
    skcnt[u] = static_cast<int64_t>(t_sk[u].size());
  }
  err = hipMemcpyAsync(base, tabs.bytes.data(), tabs.bytes.size(), hipMemcpyHostToDevice, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  if (err != hipSuccess) return err;

  // ---- the launch sequence
  const SketchJob *d_sk = reinterpret_cast<const SketchJob *>(base + o_sk);
  const OpJob *d_op = reinterpret_cast<const OpJob *>(base + o_op);
  const PivJob *d_qr = reinterpret_cast<const PivJob *>(base + o_qr);
  const InterpJob *d_in = reinterpret_cast<const InterpJob *>(base + o_in);
  const void *d_res = base + o_res;
  const int4 *d_top = reinterpret_cast<const int4 *>(base + o_top);
  const int4 *d_tqr = reinterpret_cast<const int4 *>(base + o_tqr);
  const int4 *d_tin = reinterpret_cast<const int4 *>(base + o_tin);
  const int4 *d_tres = reinterpret_cast<const int4 *>(base + o_tres);
  const int *d_qord = reinterpret_cast<const int *>(base + o_qord);
  const int qmode = qr_mode();
  const int4 *d_tsk = reinterpret_cast<const int4 *>(base + o_tsk0);
  // the sketch reduce table is appended to the sketch tables' index space
  auto sequence = [&](hipStream_t st) -> hipError_t {
    hipLaunchKernelGGL(operator_grouped_kernel, dim3(static_cast<unsigned>(t_op.size())),
                       dim3(256), 0, st, d_op, d_top);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // grouped sketch per MT bucket, then the grouped split reduce (its table
    // sits before the sketch tables: a negative offset from d_tsk)
    const int64_t red_off = (static_cast<int64_t>(o_tred) - static_cast<int64_t>(o_tsk0)) /
                            static_cast<int64_t>(sizeof(int4));
    // the bf16 planes are split over the operator's table (job, block, blocks)
    e = launch_sketch_batch(st, dtype, prec, d_sk, d_tsk, mts.data(), skoff.data(), skcnt.data(),
                            static_cast<int>(nbuck), red_off, static_cast<int64_t>(t_red.size()),
                            d_top, static_cast<int64_t>(t_op.size()), prof);
    if (e != hipSuccess) return e;
    e = qmode ? launch_pivqr_batch(st, qr_lmax.data(), qr_live.data(), kmax, d_qr, d_tqr,
                                   static_cast<int64_t>(t_qr.size()), prof, qmode)
              : launch_pivqr_jobs(st, d_qr, d_qord, count, prof);
    if (e != hipSuccess) return e;
    e = launch_interp_batch(st, kmax, d_in, d_tin, static_cast<int64_t>(t_in.size()), prof);
    if (e != hipSuccess) return e;
    return launch_residual_batch(st, dtype, d_res, d_tres, res, q, acc, prof);
  };

  if (!prof && h->batch_graph && use_graph()) {
    if (!h->cap_stream) {
      err = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
      if (err != hipSuccess) return err;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    err = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
      hipError_t e1 = sequence(h->cap_stream);
      err = hipStreamEndCapture(h->cap_stream, &graph);
      if (e1 != hipSuccess) err = e1;
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (err == hipSuccess) err = hipGraphLaunch(exec, stream);
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (err != hipSuccess) return err;
  } else {
    err = sequence(stream);
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    if (err != hipSuccess) return err;
  }
  err = hipMemcpyAsync(status, dstatus, sizeof(int) * count, hipMemcpyDeviceToHost, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  return err;
}

hipError_t run_batch(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                     const RidBatchJob *bj, int count, int q, double rank_tol, int *status,
                     RidProf *prof) {
  return run_batch_impl(h, stream, dtype, prec, bj, count, q, rank_tol, status, prof, nullptr);
}

size_t batch_ws_need(rid_handle h, rid_dtype dtype, rid_prec prec, const RidBatchJob *bj,
                     int count, int q) {
  size_t need = 0;
  (void)run_batch_impl(h, nullptr, dtype, prec, bj, count, q, 0.0, nullptr, nullptr, &need);
  return need;
}

extern "C" rid_status rid_decompose_batched(rid_handle h, hipStream_t stream, rid_dtype dtype,
                                            rid_prec prec, const rid_job *jobs, int count, int q,
                                            int max_retries, double rank_tol, int *job_status,
                                            uint64_t *seed_used) {
  if (!h || count < 0 || (count > 0 && !jobs) || q < 1 || max_retries < 0 ||
      !(rank_tol >= 0.0) || rank_tol > 1.0)
    return RID_ERR_INVALID_ARG;
  if (dtype != RID_C128 && dtype != RID_C64) return RID_ERR_INVALID_ARG;
  if (!prec_valid(prec)) return RID_ERR_INVALID_ARG;
  if (!sketch_supported(dtype, prec) || !batch_prec_supported(prec)) return RID_ERR_UNSUPPORTED;
  const size_t align = dtype == RID_C128 ? 16 : 8;
  std::vector<RidBatchJob> bj(count);
  for (int i = 0; i < count; ++i) {
    const rid_job &j = jobs[i];
    if (j.k < 1 || j.k > j.l || j.k > j.n || j.l > j.m || j.lda < j.m || j.ldp < j.k || !j.A ||
        !j.J || !j.P || !j.sigma || reinterpret_cast<uintptr_t>(j.A) % align != 0 ||
        reinterpret_cast<uintptr_t>(j.P) % 16 != 0 || j.n > 0x7FFFFFFFll)
      return RID_ERR_INVALID_ARG;
    bj[i] = RidBatchJob{j.m, j.n, j.k, j.l, j.lda, j.ldp, j.A, j.seed, j.J,
                        static_cast<double2 *>(j.P), j.sigma};
    if (!batch_job_supported(bj[i])) return RID_ERR_UNSUPPORTED;
    if (h->sketch_kind == RID_SKETCH_SRFT && j.m > 0x7FFFFFFFll) return RID_ERR_UNSUPPORTED;
  }
  if (count == 0) return RID_OK;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return RID_ERR_HIP;
  if (prev != h->device && hipSetDevice(h->device) != hipSuccess) return RID_ERR_HIP;
  std::vector<int> st(count, RID_ERR_RANK);
  std::vector<uint64_t> used(count);
  for (int i = 0; i < count; ++i) used[i] = jobs[i].seed;
  std::vector<int> pending(count);
  std::iota(pending.begin(), pending.end(), 0);
  rid_status out = RID_OK;
  for (int attempt = 0; attempt <= max_retries && !pending.empty(); ++attempt) {
    std::vector<RidBatchJob> sub;
    for (int i : pending) {
      sub.push_back(bj[i]);
      sub.back().seed = jobs[i].seed + static_cast<uint64_t>(attempt);
    }
    std::vector<int> sst(sub.size(), RID_ERR_HIP);
    // while the handle records (rid_profile), the batch is launched directly
    // with event pairs around its kernel families
    hipError_t e = run_batch(h, stream, dtype, prec, sub.data(), static_cast<int>(sub.size()), q,
                             rank_tol, sst.data(), h->prof.on ? &h->prof : nullptr);
    if (e != hipSuccess) {
      h->last_hip_error = static_cast<int>(e);
      out = RID_ERR_HIP;
      break;
    }
    std::vector<int> next;
    for (size_t u = 0; u < pending.size(); ++u) {
      st[pending[u]] = sst[u];
      used[pending[u]] = sub[u].seed;
      if (sst[u] == RID_ERR_RANK) next.push_back(pending[u]);
    }
    pending.swap(next);
  }
  if (out == RID_OK)
    for (int i = 0; i < count; ++i)
      if (st[i] != RID_OK) out = RID_ERR_RANK;
  if (job_status)
    for (int i = 0; i < count; ++i) job_status[i] = st[i];
  if (seed_used)
    for (int i = 0; i < count; ++i) seed_used[i] = used[i];
  if (prev != h->device) (void)hipSetDevice(prev);
  return out;
}

extern "C" rid_status rid_set_batch_plan(rid_handle h, int64_t sketch_rows,
                                         int64_t res_block_bytes, int ahz_cols) {
  if (!h || sketch_rows < 16 || sketch_rows > (int64_t(1) << 20) || sketch_rows % 16 != 0 ||
      res_block_bytes < (int64_t(4) << 10) || res_block_bytes > (int64_t(1) << 30) ||
      (ahz_cols != 4 && ahz_cols != 8))
    return RID_ERR_INVALID_ARG;
  h->batch_sketch_rows = sketch_rows;
  h->batch_res_block_bytes = res_block_bytes;
  h->batch_ahz_cpw = ahz_cols;
  return RID_OK;
}

extern "C" rid_status rid_get_batch_plan(rid_handle h, int64_t *sketch_rows,
                                         int64_t *res_block_bytes, int *ahz_cols) {
  if (!h) return RID_ERR_INVALID_ARG;
  if (sketch_rows) *sketch_rows = h->batch_sketch_rows;
  if (res_block_bytes) *res_block_bytes = h->batch_res_block_bytes;
  if (ahz_cols) *ahz_cols = h->batch_ahz_cpw;
  return RID_OK;
}

// Autotuner of the batched plan: candidate i pairs sketch split rows
// kRows[i] with ax block bytes kBlock[i] and ahz columns per wave kCols[i];
// one directly launched, event-timed run per candidate gives the sketch,
// ax and ahz family times of its three values (each parameter changes only
// its own family), and the fastest value of each is kept in the handle.
extern "C" rid_status rid_tune_batched(rid_handle h, hipStream_t stream, rid_dtype dtype,
                                       rid_prec prec, const rid_job *jobs, int count, int q,
                                       int64_t *sketch_rows, int64_t *res_block_bytes,
                                       int *ahz_cols) {
  static const int64_t kRows[] = {128, 256, 512, 1024, 2048, 4096};
  static const int64_t kBlock[] = {int64_t(32) << 10,  int64_t(64) << 10,  int64_t(128) << 10,
                                   int64_t(256) << 10, int64_t(512) << 10, int64_t(1024) << 10};
  static const int kCols[] = {8, 4, 8, 4, 8, 4};
  constexpr int kCand = 6;
  if (!h || count < 1 || !jobs || q < 1) return RID_ERR_INVALID_ARG;
  if (dtype != RID_C128 && dtype != RID_C64) return RID_ERR_INVALID_ARG;
  if (!prec_valid(prec)) return RID_ERR_INVALID_ARG;
  if (!sketch_supported(dtype, prec) || !batch_prec_supported(prec)) return RID_ERR_UNSUPPORTED;
  const size_t align = dtype == RID_C128 ? 16 : 8;
  std::vector<RidBatchJob> bj(count);
  for (int i = 0; i < count; ++i) {
    const rid_job &j = jobs[i];
    if (j.k < 1 || j.k > j.l || j.k > j.n || j.l > j.m || j.lda < j.m || j.ldp < j.k || !j.A ||
        !j.J || !j.P || !j.sigma || reinterpret_cast<uintptr_t>(j.A) % align != 0 ||
        reinterpret_cast<uintptr_t>(j.P) % 16 != 0 || j.n > 0x7FFFFFFFll)
      return RID_ERR_INVALID_ARG;
    bj[i] = RidBatchJob{j.m, j.n, j.k, j.l, j.lda, j.ldp, j.A, j.seed, j.J,
                        static_cast<double2 *>(j.P), j.sigma};
    if (!batch_job_supported(bj[i])) return RID_ERR_UNSUPPORTED;
  }
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return RID_ERR_HIP;
  if (prev != h->device && hipSetDevice(h->device) != hipSuccess) return RID_ERR_HIP;
  const int64_t keep_rows = h->batch_sketch_rows, keep_block = h->batch_res_block_bytes;
  const int keep_cols = h->batch_ahz_cpw;
  std::vector<int> st(count);
  double best_sk = 1e300, best_ax = 1e300, best_ahz = 1e300;
  int64_t pick_rows = keep_rows, pick_block = keep_block;
  int pick_cols = keep_cols;
  rid_status out = RID_OK;
  RidProf prof;
  for (int c = -1; c < kCand && out == RID_OK; ++c) {  // c = -1: warm-up, untimed
    h->batch_sketch_rows = c < 0 ? keep_rows : kRows[c];
    h->batch_res_block_bytes = c < 0 ? keep_block : kBlock[c];
    h->batch_ahz_cpw = c < 0 ? keep_cols : kCols[c];
    prof.on = true;
    prof.used = 0;
    prof.recs.clear();
    hipError_t e = run_batch(h, stream, dtype, prec, bj.data(), count, q, 0.0, st.data(), &prof);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    double fam[RID_KERNEL_COUNT] = {0.0};
    for (const auto &r : prof.recs) {
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, prof.pool[r.second], prof.pool[r.second + 1]);
      fam[r.first] += ms;
    }
    if (e != hipSuccess) {
      h->last_hip_error = static_cast<int>(e);
      out = RID_ERR_HIP;
      break;
    }
    if (c < 0) continue;
    if (fam[RID_KERNEL_SKETCH] < best_sk) {
      best_sk = fam[RID_KERNEL_SKETCH];
      pick_rows = kRows[c];
    }
    if (fam[RID_KERNEL_AX] < best_ax) {
      best_ax = fam[RID_KERNEL_AX];
      pick_block = kBlock[c];
    }
    if (fam[RID_KERNEL_AHZ] < best_ahz) {
      best_ahz = fam[RID_KERNEL_AHZ];
      pick_cols = kCols[c];
    }
  }
  for (hipEvent_t ev : prof.pool) (void)hipEventDestroy(ev);
  h->batch_sketch_rows = out == RID_OK ? pick_rows : keep_rows;
  h->batch_res_block_bytes = out == RID_OK ? pick_block : keep_block;
  h->batch_ahz_cpw = out == RID_OK ? pick_cols : keep_cols;
  if (sketch_rows) *sketch_rows = h->batch_sketch_rows;
  if (res_block_bytes) *res_block_bytes = h->batch_res_block_bytes;
  if (ahz_cols) *ahz_cols = h->batch_ahz_cpw;
  if (prev != h->device) (void)hipSetDevice(prev);
  return out;
}
