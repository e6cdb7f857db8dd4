// server.hip -- continuous batching of ID requests on one device
// (rid_server_*).  Host code only: the lanes drive the same entry points a
// caller would (rid_decompose_batched for a batch, rid_decompose for a job
// alone), each lane on its own handle and non-blocking stream.
//
// Admission is by device footprint.  The budget covers the data of the
// admitted requests (bytes(A) + fill scratch + outputs) and every device
// workspace the lanes hold: a lane's handle keeps its workspace, and the
// superseded ones, between requests, and all of it stays counted while it
// is held.  A group is admitted on a lane when its data plus the workspace
// the lane would allocate for it (exact: the single-ID workspace for a job
// alone, the batch planner's figure for a batch) fits beside what is
// counted already.  A batch lane takes the oldest small request and every
// later queued small request with the same (dtype, prec, q, max_retries,
// rank_tol) that still fits, up to max_batch, so requests that arrived while
// the previous batch ran join the next one; big lanes take one big request
// each.  When a lane's group does not fit, every idle lane that holds a
// workspace frees it (hipFree, which waits for the device: this happens
// only when the budget is short); a request whose data and workspace exceed
// the budget alone is refused at submission, so a waiting group fits once
// the work ahead of it is done and the idle lanes have let go.  All lanes
// run at once, so a long big job does not hold up the small ones: lane
// threads use the short-workgroup plans (a workgroup of a big ID frees its
// CU slots within about a millisecond), and otherwise a lane never
// synchronises the whole device (workspaces grow without freeing, streams
// are non-blocking, and lanes launch batches directly rather than capturing
// graphs).
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
  int64_t data;       // bytes(A) + fill scratch + outputs
  int64_t footprint;  // data + the workspace of the job run alone
  double t[4];        // arrival, admission, A in place, done
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
  // admitted data + reserved workspace growth + workspace the lanes hold
  int64_t committed = 0, peak = 0;
  int blocked = 0;  // lanes whose next group does not fit
  int64_t pending = 0;  // submitted, not yet done
  int64_t completed = 0, batches = 0;
  uint64_t next_ticket = 1;
  bool stop = false;

  struct Lane {
    rid_handle h = nullptr;
    hipStream_t st = nullptr;
    bool big = false;
    int64_t held = 0;      // workspace bytes the handle holds (counted)
    int64_t reserved = 0;  // workspace growth reserved for the running group
  };
  std::vector<Lane> lanes;
  std::vector<std::thread> threads;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  bool fits(int64_t bytes) const { return committed + bytes <= cfg.hbm_budget; }
};

namespace {

void finish(rid_server s, rid_server_ctx::Lane &ln, std::vector<SrvJob> &jobs,
            const std::vector<int> &status, const std::vector<uint64_t> &used) {
  const double t = s->now();
  for (size_t i = 0; i < jobs.size(); ++i) {
    jobs[i].t[3] = t;
    if (s->done) s->done(s->user, jobs[i].ticket, status[i], used[i], jobs[i].t);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  for (const SrvJob &j : jobs) s->committed -= j.data;
  // the reservation becomes what the handle now holds (at most as much)
  const int64_t held = static_cast<int64_t>(ws_held_bytes(ln.h));
  s->committed += held - ln.held - ln.reserved;
  ln.held = held;
  ln.reserved = 0;
  if (s->committed > s->peak) s->peak = s->committed;
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
  finish(s, ln, jobs, status, used);
}

// Workspace a lane's handle needs for one request alone (rid_decompose),
// with the lanes' short-workgroup plans whatever the calling thread.
size_t single_need(const rid_request &r) {
  const bool prev = rid_tl_short_blocks;
  rid_tl_short_blocks = true;
  const size_t ws = decomp_ws_bytes(r.dtype, r.prec, r.m, r.n, r.k, r.l, r.q);
  rid_tl_short_blocks = prev;
  return ws;
}

int64_t data_of(const rid_request &r) {
  const int64_t es = r.dtype == RID_C128 ? 16 : 8;
  return r.m * r.n * es + r.fill_bytes + r.k * r.n * 16 + r.k * 8 + 8;
}

// Workspace growth of lane ln for a group: a group that the fill callbacks
// reduce to one job runs alone, a larger one as a batch (whose subsets need
// no more), so the reservation covers both.  Host planning only.
int64_t group_growth(const rid_server_ctx::Lane &ln, const std::vector<const SrvJob *> &g) {
  size_t need = 0;
  for (const SrvJob *j : g) need = std::max(need, single_need(j->req));
  if (g.size() > 1) {
    std::vector<RidBatchJob> bj;
    for (const SrvJob *j : g) {
      const rid_request &r = j->req;
      bj.push_back(RidBatchJob{r.m, r.n, r.k, r.l, r.m, r.k, nullptr, r.seed, nullptr, nullptr,
                               nullptr});
    }
    const rid_request &r0 = g[0]->req;
    need = std::max(need, batch_ws_need(ln.h, r0.dtype, r0.prec, bj.data(),
                                        static_cast<int>(bj.size()), r0.q));
  }
  return static_cast<int64_t>(ws_grow_bytes(ln.h, need));
}

// Under the lock: the next group of queue q for lane ln if it fits (then it
// leaves the queue and is counted), else false.  The group is the oldest
// request and later ones of its kind, while their data fit; then halved
// until data and workspace growth fit together.
bool take_group(rid_server s, rid_server_ctx::Lane &ln, std::deque<SrvJob> &q,
                std::vector<SrvJob> &group) {
  const int cap = ln.big ? 1 : s->cfg.max_batch;
  const rid_request key = q.front().req;
  std::vector<std::deque<SrvJob>::iterator> pick;
  int64_t data = 0;
  for (auto it = q.begin(); it != q.end() && static_cast<int>(pick.size()) < cap; ++it) {
    if (!same_group(key, it->req)) continue;
    if (!s->fits(data + it->data)) break;  // keep arrival order within a group
    pick.push_back(it);
    data += it->data;
  }
  while (!pick.empty()) {
    std::vector<const SrvJob *> g;
    for (auto it : pick) g.push_back(&*it);
    const int64_t growth = group_growth(ln, g);
    if (s->fits(data + growth)) {
      s->committed += data + growth;
      ln.reserved = growth;
      if (s->committed > s->peak) s->peak = s->committed;
      for (auto it : pick) group.push_back(*it);
      for (auto r = pick.rbegin(); r != pick.rend(); ++r) q.erase(*r);
      return true;
    }
    if (pick.size() == 1) break;
    const size_t keep = pick.size() / 2;
    for (size_t i = keep; i < pick.size(); ++i) data -= pick[i]->data;
    pick.resize(keep);
  }
  return false;
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
      bool waiting = false;  // counted in s->blocked
      for (;;) {
        if (!q.empty() && take_group(s, ln, q, group)) break;
        const bool stuck = !q.empty();
        if (stuck != waiting) {
          s->blocked += stuck ? 1 : -1;
          waiting = stuck;
          s->cv.notify_all();
        }
        if (q.empty() && s->stop) return;  // stop with nothing left
        if (s->blocked > 0 && ln.held > 0) {
          // an idle lane lets its workspace go while some group cannot fit
          const int64_t held = ln.held;
          lk.unlock();
          release_ws(ln.h);
          lk.lock();
          s->committed -= held;
          ln.held = 0;
          s->cv.notify_all();
          continue;
        }
        s->cv.wait(lk);
      }
      if (waiting) {
        --s->blocked;
        s->cv.notify_all();
      }
    }
    run_group(s, ln, group);
  }
}

// The footprint of a request run alone on a lane that holds nothing.
int64_t footprint_of(const rid_request &r) {
  const size_t ws = single_need(r);
  return data_of(r) + static_cast<int64_t>((ws + 4095) & ~size_t(4095));
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
  j.data = data_of(r);
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
