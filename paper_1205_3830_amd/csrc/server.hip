// server.hip -- continuous batching of ID requests on one device
// (rid_server_*).  Host code only: the lanes drive the same entry points a
// caller would (rid_decompose_batched for a batch, rid_decompose for a job
// alone), each lane on its own handle and non-blocking stream.
//
// Admission is by device footprint: a request waits in its class queue
// (small or big) until bytes(A) + fill scratch + outputs + the workspace
// of its shape fit the budget beside the jobs already admitted.  A batch
// lane takes the oldest small request and every later queued small request
// with the same (dtype, prec, q, max_retries, rank_tol) that still fits, up
// to max_batch, so requests that arrived while the previous batch ran join
// the next one.  Big lanes take one big request each.  All lanes run at
// once, so a long big job does not hold up the small ones: lane threads use
// the short-workgroup plans (a workgroup of a big ID frees its CU slots
// within about a millisecond), and a lane never synchronises the whole
// device (workspaces grow without freeing, streams are non-blocking, and
// lanes launch batches directly rather than capturing graphs).
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "rid_internal.hpp"

namespace {

struct SrvJob {
  uint64_t ticket;
  rid_request req;
  int64_t footprint;
  double t[4];  // arrival, admission, A in place, done
};

bool same_group(const rid_request &a, const rid_request &b) {
  return a.dtype == b.dtype && a.prec == b.prec && a.q == b.q && a.max_retries == b.max_retries &&
         a.rank_tol == b.rank_tol;
}

}  // namespace

struct rid_server_ctx {
  int device = 0;
  rid_server_config cfg{};
  rid_admit_fn admit = nullptr;
  rid_done_fn done = nullptr;
  void *user = nullptr;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv;       // queue or budget changed
  std::condition_variable idle_cv;  // a job finished
  std::deque<SrvJob> small_q, big_q;
  int64_t committed = 0, peak = 0;
  int64_t pending = 0;  // submitted, not yet done
  int64_t completed = 0, batches = 0;
  uint64_t next_ticket = 1;
  bool stop = false;

  struct Lane {
    rid_handle h = nullptr;
    hipStream_t st = nullptr;
    bool big = false;
  };
  std::vector<Lane> lanes;
  std::vector<std::thread> threads;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  bool fits(int64_t fp) const { return committed + fp <= cfg.hbm_budget; }
};

namespace {

void finish(rid_server s, std::vector<SrvJob> &jobs, const std::vector<int> &status,
            const std::vector<uint64_t> &used) {
  const double t = s->now();
  for (size_t i = 0; i < jobs.size(); ++i) {
    jobs[i].t[3] = t;
    if (s->done) s->done(s->user, jobs[i].ticket, status[i], used[i], jobs[i].t);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  for (const SrvJob &j : jobs) s->committed -= j.footprint;
  s->pending -= static_cast<int64_t>(jobs.size());
  s->completed += static_cast<int64_t>(jobs.size());
  s->cv.notify_all();
  s->idle_cv.notify_all();
}

// Admission of the requests in `jobs` (callbacks), then one run.
void run_group(rid_server s, rid_server_ctx::Lane &ln, std::vector<SrvJob> &jobs) {
  const size_t cnt = jobs.size();
  std::vector<rid_job> rj(cnt);
  std::vector<int> status(cnt, RID_OK);
  std::vector<uint64_t> used(cnt);
  std::vector<size_t> live;
  for (size_t i = 0; i < cnt; ++i) {
    const rid_request &r = jobs[i].req;
    jobs[i].t[1] = s->now();
    used[i] = r.seed;
    rj[i] = rid_job{r.m, r.n, r.k, r.l, nullptr, 0, r.seed, nullptr, nullptr, 0, nullptr};
    const int rc = s->admit ? s->admit(s->user, jobs[i].ticket, ln.st, &rj[i]) : 1;
    if (rc != 0) {
      status[i] = RID_ERR_INVALID_ARG;
    } else {
      live.push_back(i);
    }
  }
  hipError_t e = hipStreamSynchronize(ln.st);
  const double tf = s->now();
  for (size_t i = 0; i < cnt; ++i) jobs[i].t[2] = tf;
  if (e != hipSuccess) {
    for (size_t i : live) status[i] = RID_ERR_HIP;
    live.clear();
  }
  if (live.size() == 1) {
    const size_t i = live[0];
    const rid_request &r = jobs[i].req;
    const rid_job &j = rj[i];
    uint64_t u = r.seed;
    status[i] = rid_decompose(ln.h, ln.st, r.dtype, r.prec, j.m, j.n, j.k, j.l, j.A, j.lda, j.seed,
                              r.q, r.max_retries, r.rank_tol, j.J, j.P, j.ldp, j.sigma, &u);
    used[i] = u;
  } else if (live.size() > 1) {
    const rid_request &r = jobs[live[0]].req;
    std::vector<rid_job> sub;
    for (size_t i : live) sub.push_back(rj[i]);
    std::vector<int> st(sub.size(), RID_ERR_HIP);
    std::vector<uint64_t> u(sub.size());
    const rid_status all =
        rid_decompose_batched(ln.h, ln.st, r.dtype, r.prec, sub.data(), static_cast<int>(sub.size()),
                              r.q, r.max_retries, r.rank_tol, st.data(), u.data());
    for (size_t v = 0; v < live.size(); ++v) {
      const size_t i = live[v];
      if (all == RID_OK || all == RID_ERR_RANK) {
        status[i] = st[v];
        used[i] = u[v];
      } else {
        status[i] = all;
      }
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->batches;
  }
  finish(s, jobs, status, used);
}

void lane_main(rid_server s, int id) {
  rid_server_ctx::Lane &ln = s->lanes[id];
  (void)hipSetDevice(s->device);
  rid_tl_short_blocks = true;  // share the device with the other lanes
  for (;;) {
    std::vector<SrvJob> group;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      std::deque<SrvJob> &q = ln.big ? s->big_q : s->small_q;
      s->cv.wait(lk, [&] { return (!q.empty() && s->fits(q.front().footprint)) || (s->stop && q.empty()); });
      if (q.empty()) return;  // stop with nothing left
      const int cap = ln.big ? 1 : s->cfg.max_batch;
      const rid_request key = q.front().req;
      for (auto it = q.begin(); it != q.end() && static_cast<int>(group.size()) < cap;) {
        if (!same_group(key, it->req)) {
          ++it;
          continue;
        }
        if (!s->fits(it->footprint)) break;  // keep arrival order within a group
        s->committed += it->footprint;
        group.push_back(*it);
        it = q.erase(it);
      }
      if (s->committed > s->peak) s->peak = s->committed;
    }
    run_group(s, ln, group);
  }
}

// sized with the lanes' short-workgroup plans, whatever the calling thread
int64_t footprint_of(const rid_request &r) {
  const int64_t es = r.dtype == RID_C128 ? 16 : 8;
  const bool prev = rid_tl_short_blocks;
  rid_tl_short_blocks = true;
  const int64_t ws =
      static_cast<int64_t>(decomp_ws_bytes(r.dtype, r.prec, r.m, r.n, r.k, r.l, r.q));
  rid_tl_short_blocks = prev;
  return r.m * r.n * es + r.fill_bytes + r.k * r.n * 16 + r.k * 8 + 8 + ws;
}

}  // namespace

extern "C" {

rid_status rid_server_create(rid_server *out, int device, const rid_server_config *cfg,
                             rid_admit_fn admit, rid_done_fn done, void *ctx) {
  if (!out) return RID_ERR_INVALID_ARG;
  *out = nullptr;
  if (!cfg || !admit || cfg->hbm_budget <= 0 || cfg->big_bytes <= 0 || cfg->big_lanes < 0 ||
      cfg->big_lanes > 64 || cfg->batch_lanes < 1 || cfg->batch_lanes > 64 || cfg->max_batch < 1)
    return RID_ERR_INVALID_ARG;
  rid_server s = new (std::nothrow) rid_server_ctx();
  if (!s) return RID_ERR_NOMEM;
  s->device = device;
  s->cfg = *cfg;
  s->admit = admit;
  s->done = done;
  s->user = ctx;
  s->t0 = std::chrono::steady_clock::now();
  const int nl = cfg->batch_lanes + cfg->big_lanes;
  s->lanes.resize(nl);
  rid_status st = RID_OK;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) st = RID_ERR_HIP;
  for (int i = 0; i < nl && st == RID_OK; ++i) {
    s->lanes[i].big = i >= cfg->batch_lanes;
    st = rid_create(&s->lanes[i].h, device);
    // lanes launch batches directly: a capture on one lane thread must not
    // overlap the calls other lane threads (and the fill callbacks) make
    if (st == RID_OK) s->lanes[i].h->batch_graph = false;
    if (st == RID_OK) {
      if (hipSetDevice(device) != hipSuccess ||
          hipStreamCreateWithFlags(&s->lanes[i].st, hipStreamNonBlocking) != hipSuccess)
        st = RID_ERR_HIP;
    }
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  if (st != RID_OK) {
    for (auto &ln : s->lanes) {
      if (ln.st) (void)hipStreamDestroy(ln.st);
      if (ln.h) (void)rid_destroy(ln.h);
    }
    delete s;
    return st;
  }
  for (int i = 0; i < nl; ++i) s->threads.emplace_back(lane_main, s, i);
  *out = s;
  return RID_OK;
}

rid_status rid_server_submit(rid_server s, const rid_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return RID_ERR_INVALID_ARG;
  const rid_request &r = *req;
  if (r.k < 1 || r.k > r.l || r.k > r.n || r.l > r.m || r.q < 1 || r.max_retries < 0 ||
      r.fill_bytes < 0 || !(r.rank_tol >= 0.0) || r.rank_tol > 1.0 || r.n > 0x7FFFFFFFll)
    return RID_ERR_INVALID_ARG;
  if (r.dtype != RID_C128 && r.dtype != RID_C64) return RID_ERR_INVALID_ARG;
  if (!prec_valid(r.prec)) return RID_ERR_INVALID_ARG;
  if (!sketch_supported(r.dtype, r.prec) || !pivqr_supported(r.l) || !interp_supported(r.k))
    return RID_ERR_UNSUPPORTED;
  const int64_t es = r.dtype == RID_C128 ? 16 : 8;
  const bool big = s->cfg.big_lanes > 0 && r.m * r.n * es >= s->cfg.big_bytes;
  if (!big) {
    RidBatchJob bj{r.m, r.n, r.k, r.l, r.m, r.k, nullptr, r.seed, nullptr, nullptr, nullptr};
    if (!batch_job_supported(bj) || !batch_prec_supported(r.prec)) return RID_ERR_UNSUPPORTED;
  }
  SrvJob j{};
  j.req = r;
  j.footprint = footprint_of(r);
  if (j.footprint > s->cfg.hbm_budget) return RID_ERR_NOMEM;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return RID_ERR_INVALID_ARG;
    j.ticket = s->next_ticket++;
    j.t[0] = s->now();
    (big ? s->big_q : s->small_q).push_back(j);
    ++s->pending;
    *ticket = j.ticket;
  }
  s->cv.notify_all();
  return RID_OK;
}

rid_status rid_server_drain(rid_server s) {
  if (!s) return RID_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->idle_cv.wait(lk, [&] { return s->pending == 0; });
  return RID_OK;
}

rid_status rid_server_stats(rid_server s, int64_t *peak_bytes, int64_t *completed,
                            int64_t *batches) {
  if (!s) return RID_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (peak_bytes) *peak_bytes = s->peak;
  if (completed) *completed = s->completed;
  if (batches) *batches = s->batches;
  return RID_OK;
}

rid_status rid_server_destroy(rid_server s) {
  if (!s) return RID_ERR_INVALID_ARG;
  (void)rid_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto &t : s->threads) t.join();
  for (auto &ln : s->lanes) {
    if (ln.st) (void)hipStreamDestroy(ln.st);
    if (ln.h) (void)rid_destroy(ln.h);
  }
  delete s;
  return RID_OK;
}

}  // extern "C"
