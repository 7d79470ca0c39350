// Serving engine: continuous batching of range queries interleaved with
// stream appends, on one device.
//
// Callers submit queries and appends from any thread and get tickets; a
// scheduler thread owned by the tree admits work and issues it:
//   * appends are staged in submission order and committed (leaf Tucker of
//     each completed block, then its merges, level by level) on the append
//     lane's stream, as many blocks per commit as have arrived;
//   * a query sees the tree as of its submission (read-your-writes: the
//     committed horizon T_c of every append submitted before it).  Completed
//     nodes never change (Alg. "insert" only fills placeholders), so a query
//     reads a consistent snapshot while later appends add nodes; it is
//     admitted once every node of its hit set (Recall at its snapshot) has
//     been written (commits record an event per tree level, so a query can
//     start once the levels it needs are done, before the commit's upper
//     levels), and a query away from the latest appends never waits;
//   * queries are grouped into three size classes by their largest
//     eigenproblem.  Each class has a job ring in host memory that the
//     device maps, and a stitch launch on the class's stream whose
//     workgroups claim published jobs one at a time as they become free
//     (a workgroup is a job slot).  A query is admitted, in arrival order, as
//     soon as its class's ring has a free entry and the class's workspace
//     has room for it (first fit): it joins the work already running on
//     the device instead of waiting for a batch to finish.  A launch ends by
//     itself when its class has been idle for 2 ms, or at 20 ms of age (so
//     the class's hardware queue also serves other streams' work); the
//     scheduler launches again whenever published jobs are waiting.
// A query's result depends only on its range and snapshot: the kernel
// variant is a function of the query's own eigenproblem size, so a query
// returns the same bits alone and in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "tk_host.hpp"

namespace tk {

namespace {

constexpr int kClasses = 3;
constexpr uint64_t kRingIdleTicks = 200000;    // 2 ms of the device's 100 MHz clock
constexpr uint64_t kRingLifeTicks = 2000000;   // 20 ms: streams outnumber the hardware queues, so a
                                               // queue that a class's launch holds frees up this often
                                               // for the append commits queued behind it

double now_us(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

enum { REQ_QUEUED = 0, REQ_RUNNING = 1, REQ_DONE = 2, REQ_FAILED = 3 };

struct Request {
  uint64_t ticket = 0;
  int kind = 0;  // 0 query, 1 append
  int cls = 0;
  int64_t ts = 0, te = 0, Tb = 0;
  tk_result* res = nullptr;
  Job job{};
  std::vector<Hit> hits;
  std::vector<float> data;          // host append: a copy of the slice
  const float* dev_slice = nullptr;  // device append
  double t_submit = 0, t_launch = 0, t_done = 0;
  int state = REQ_QUEUED;
  int need = 0;  // size of the query's largest eigenproblem
  int64_t seq = -1, slot = -1, ws_off = -1;  // ring position and workspace of an admitted query
  int64_t Tb_need = 0;  // committed blocks its hit nodes need: max over hits of (index + 1) 2^level
};

struct ClassLane {
  Lane lane;  // stream, workspace, ring head counter
  int n_lds = 0;
  int threads = 64;
  int lds_doubles = 0;
  int grid = 0;  // job slots: workgroups of the class's launch
  int64_t ws_budget = 0;
  std::deque<Request*> pending;
  std::vector<Request*> inflight;  // admitted, not done
  // the job ring (pinned host memory, mapped on the device)
  void* host = nullptr;
  int64_t slots = 0;
  RingHdr* hdr = nullptr;
  Job* jobs = nullptr;
  Hit* hits = nullptr;  // host-planned hit sets (fixed-block queries); Recall writes its own
  double* stats = nullptr;
  int64_t* done = nullptr;
  StitchRing dring{};
  Hit* dhits = nullptr;
  double* dstats = nullptr;
  std::vector<Request*> slot_req;
  int64_t published = 0;
  std::vector<std::pair<int64_t, int64_t>> allocs;  // workspace in use: (offset, bytes), by offset
  hipEvent_t kev = nullptr;
  bool launched = false;
};

}  // namespace

struct Server {
  tk_tree* t = nullptr;
  tk_serve_config cfg{};
  std::chrono::steady_clock::time_point t0;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;       // new work or stop
  std::condition_variable done_cv;  // a request finished
  bool stop = false;
  bool failed = false;
  std::vector<Request*> reqs;  // by ticket - 1
  std::deque<Request*> inbox;
  int64_t T_logical = 0;  // slices submitted
  int64_t outstanding = 0;
  tk_serve_stats stats{};
  // engine-side state (scheduler thread only)
  Lane alane;
  std::deque<Request*> apending;
  std::vector<Request*> ainflight;
  hipEvent_t aev = nullptr;
  bool abusy = false;
  int64_t rows_staged = 0;  // rows of the current partial block in the staging buffer
  int64_t Tb_issued = 0;    // blocks whose commit has been issued
  int64_t Tb_done = 0;      // blocks whose commit has completed
  hipEvent_t commit_ev = nullptr;
  // per-level progress of the commit in flight: its level-k nodes are
  // written once lev_ev[k] has passed; Tb_lvl[k] blocks have every node of
  // levels <= k written (a query waits only for the nodes of its hit set)
  hipEvent_t lev_ev[MAXLEV] = {};
  int64_t Tb_lvl[MAXLEV] = {};
  int lev_count = 0, lev_next = 0;
  int64_t lev_b1 = 0;
  ClassLane cl[kClasses];
  int bounds[kClasses] = {0, 0, 0};  // class c takes eigenproblems <= bounds[c]
};

namespace {

tk_status serve_fail(Server* s, tk_status st) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->failed = true;
  for (Request* r : s->reqs)
    if (r->state < REQ_DONE) r->state = REQ_FAILED;
  s->outstanding = 0;
  s->done_cv.notify_all();
  return st;
}

void finish(Server* s, Request* r, int state) {
  r->t_done = now_us(s->t0);
  std::lock_guard<std::mutex> lk(s->mu);
  r->state = state;
  r->data.clear();
  r->data.shrink_to_fit();
  r->hits.clear();
  r->hits.shrink_to_fit();
  s->outstanding -= 1;
  s->stats.completed += 1;
  s->done_cv.notify_all();
}

int class_of(const Server* s, int need) {
  for (int c = 0; c < kClasses; ++c)
    if (need <= s->bounds[c]) return c;
  return kClasses - 1;
}

// Stage pending appends and commit the blocks they complete.
tk_status issue_appends(Server* s) {
  tk_tree* t = s->t;
  if (s->abusy || s->apending.empty()) return TK_OK;
  const int64_t ell = t->ell;
  const int64_t cap_rows = int64_t(s->cfg.max_commit_blocks) * ell;
  float* stage = reinterpret_cast<float*>(s->alane.xbuf.p);
  const int64_t se = t->slice_elems;
  const double tl = now_us(s->t0);
  while (!s->apending.empty() && s->rows_staged < cap_rows) {
    Request* r = s->apending.front();
    s->apending.pop_front();
    const float* src = r->kind == 1 && r->dev_slice ? r->dev_slice : r->data.data();
    TK_HIP(t, hipMemcpyAsync(stage + s->rows_staged * se, src, size_t(se) * 4,
                             r->dev_slice ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->alane.stream));
    r->t_launch = tl;
    r->state = REQ_RUNNING;
    s->ainflight.push_back(r);
    s->rows_staged += 1;
  }
  const int64_t nb = s->rows_staged / ell;
  if (nb > 0) {
    const int64_t b1 = t->Tb + nb;
    tk_status st = commit_blocks(t, &s->alane, nb, stage, s->lev_ev, MAXLEV);
    if (st) return st;
    s->lev_count = root_level(b1) + 1;
    s->lev_next = 0;
    s->lev_b1 = b1;
    t->T += nb * ell;
    const int64_t rem = s->rows_staged - nb * ell;
    if (rem > 0)  // keep the partial block's rows at the front (no overlap: rem < ell <= nb ell)
      TK_HIP(t, hipMemcpyAsync(stage, stage + nb * ell * se, size_t(rem * se) * 4, hipMemcpyDeviceToDevice,
                               s->alane.stream));
    s->rows_staged = rem;
    s->Tb_issued = t->Tb;
    TK_HIP(t, hipEventRecord(s->commit_ev, s->alane.stream));
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.commits += 1;
  }
  TK_HIP(t, hipEventRecord(s->aev, s->alane.stream));
  s->abusy = true;
  return TK_OK;
}

// First fit of bytes in the class's workspace; false if no gap is large enough.
bool ws_alloc(ClassLane& c, int64_t bytes, int64_t* off) {
  int64_t at = 0;
  size_t k = 0;
  for (; k < c.allocs.size(); ++k) {
    if (c.allocs[k].first - at >= bytes) break;
    at = align256(c.allocs[k].first + c.allocs[k].second);
  }
  if (k == c.allocs.size() && c.ws_budget - at < bytes) return false;
  c.allocs.insert(c.allocs.begin() + k, {at, bytes});
  *off = at;
  return true;
}

void ws_free(ClassLane& c, int64_t off) {
  for (size_t k = 0; k < c.allocs.size(); ++k)
    if (c.allocs[k].first == off) {
      c.allocs.erase(c.allocs.begin() + k);
      return;
    }
}

bool launch_running(tk_tree* t, ClassLane& c, tk_status* st) {
  *st = TK_OK;
  if (!c.launched) return false;
  const hipError_t e = hipEventQuery(c.kev);
  if (e == hipErrorNotReady) return true;
  if (e != hipSuccess) *st = fail_dev(t, e, "query launch");
  c.launched = false;
  return false;
}

// Admit waiting queries of class c into its ring (arrival order) while ring
// entries and workspace last, and make sure a launch is running while
// admitted queries are not done.
tk_status issue_queries(Server* s, ClassLane& c) {
  tk_tree* t = s->t;
  const double tl = now_us(s->t0);
  int64_t admitted = 0;
  // in arrival order; a query whose hit nodes are not all committed yet
  // (its range reaches the latest appends) waits without holding back the
  // queries behind it
  for (auto it = c.pending.begin(); it != c.pending.end();) {
    Request* r = *it;
    bool ready = r->Tb_need <= s->Tb_done;
    if (!ready) {  // the commit in flight may already have written the levels it needs
      ready = true;
      for (const Hit& x : r->hits)
        if (((x.index + 1) << x.level) > s->Tb_lvl[x.level]) {
          ready = false;
          break;
        }
    }
    if (!ready) {
      ++it;
      continue;
    }
    const int64_t slot = c.published % c.slots;
    if (c.slot_req[size_t(slot)]) break;  // the ring is full
    int64_t off = 0;
    if (!ws_alloc(c, r->job.ws_bytes, &off)) break;  // no room in the workspace yet
    it = c.pending.erase(it);
    Job jb = r->job;
    jb.hit0 = int32_t(slot * MAXHITS);
    jb.ws_off = off;
    jb.stats = c.dstats + STAT_COUNT * slot;
    c.jobs[slot] = jb;
    std::memcpy(c.hits + slot * MAXHITS, r->hits.data(), size_t(r->job.s) * sizeof(Hit));
    __atomic_store_n(&c.done[slot], int64_t(0), __ATOMIC_RELAXED);
    r->seq = c.published;
    r->slot = slot;
    r->ws_off = off;
    r->t_launch = tl;
    r->state = REQ_RUNNING;
    c.slot_req[size_t(slot)] = r;
    c.inflight.push_back(r);
    c.published += 1;
    __atomic_store_n(&c.hdr->tail, c.published, __ATOMIC_RELEASE);  // publish
    admitted += 1;
  }
  if (admitted) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (int64_t(c.inflight.size()) > s->stats.max_batch_seen) s->stats.max_batch_seen = int64_t(c.inflight.size());
  }
  if (c.inflight.empty()) return TK_OK;
  tk_status st = TK_OK;
  if (launch_running(t, c, &st) || st) return st;
  // every job claimed by an ended launch is done, so the waiting ones need a new launch
  StitchArgs a = stitch_args(t, t->q_max_iter, t->q_tol);
  a.ring = c.dring;
  a.hits = c.dhits;
  a.jobs = nullptr;
  a.ws = c.lane.ws[0].p;
  a.n_jobs = c.grid;
  a.queue = nullptr;
  a.n_lds = c.n_lds;
  a.lds_doubles = c.lds_doubles;
  TK_HIP(t, launch_stitch(a, c.grid, size_t(c.lds_doubles) * 8, c.threads, c.lane.stream));
  TK_HIP(t, hipEventRecord(c.kev, c.lane.stream));
  c.launched = true;
  std::lock_guard<std::mutex> lk(s->mu);
  s->stats.batches += 1;
  return TK_OK;
}

tk_status poll_completions(Server* s, bool* progress) {
  tk_tree* t = s->t;
  while (s->lev_next < s->lev_count) {  // levels of the commit in flight, in order
    const hipError_t e = hipEventQuery(s->lev_ev[s->lev_next]);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return fail_dev(t, e, "append commit level");
    s->Tb_lvl[s->lev_next] = s->lev_b1;
    s->lev_next += 1;
    *progress = true;
  }
  if (s->abusy) {
    const hipError_t e = hipEventQuery(s->aev);
    if (e == hipSuccess) {
      s->abusy = false;
      s->Tb_done = s->Tb_issued;
      for (int k = 0; k < MAXLEV; ++k) s->Tb_lvl[k] = std::max(s->Tb_lvl[k], s->Tb_done);
      s->lev_next = s->lev_count;
      for (Request* r : s->ainflight) finish(s, r, REQ_DONE);
      s->ainflight.clear();
      *progress = true;
    } else if (e != hipErrorNotReady) {
      return fail_dev(t, e, "append commit");
    }
  }
  for (ClassLane& c : s->cl) {
    if (c.inflight.empty()) continue;
    size_t keep = 0;
    for (size_t i = 0; i < c.inflight.size(); ++i) {
      Request* r = c.inflight[i];
      if (__atomic_load_n(&c.done[r->slot], __ATOMIC_ACQUIRE) != r->seq + 1) {
        c.inflight[keep++] = r;
        continue;
      }
      *progress = true;
      const double* st = c.stats + STAT_COUNT * r->slot;
      int state = REQ_DONE;
      if (st[STAT_STATUS] != 0.0) {
        set_error(t, job_status_msg(st[STAT_STATUS]));
        state = REQ_FAILED;
      }
      tk_result& o = *r->res;
      for (int m = 0; m < TK_MAX_MODES; ++m) o.ranks_eff[m] = m < t->p ? r->job.rq[m] : 0;
      o.fit = st[STAT_FIT];
      o.err_model = st[STAT_ERR];
      o.norm_ytilde = st[STAT_NORM];
      o.sweeps = int32_t(st[STAT_SWEEPS]);
      o.converged = int32_t(st[STAT_CONV]);
      o.n_hits = r->job.s;
      ws_free(c, r->ws_off);
      c.slot_req[size_t(r->slot)] = nullptr;
      finish(s, r, state);
    }
    c.inflight.resize(keep);
    // a launch that ended with a device error
    tk_status st = TK_OK;
    (void)launch_running(t, c, &st);
    if (st) return st;
  }
  return TK_OK;
}

void engine(Server* s) {
  tk_tree* t = s->t;
  (void)hipSetDevice(t->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      const bool idle = !s->abusy && s->apending.empty() && s->inbox.empty() &&
                        std::all_of(s->cl, s->cl + kClasses, [](const ClassLane& c) {
                          return c.inflight.empty() && c.pending.empty();
                        });
      if (idle) {
        if (s->stop) break;
        s->cv.wait(lk, [&] { return s->stop || !s->inbox.empty(); });
      }
      while (!s->inbox.empty()) {
        Request* r = s->inbox.front();
        s->inbox.pop_front();
        if (r->kind == 1) s->apending.push_back(r);
        else s->cl[r->cls].pending.push_back(r);
      }
    }
    bool progress = false;
    tk_status st = poll_completions(s, &progress);
    if (!st) st = issue_appends(s);
    for (int c = 0; c < kClasses && !st; ++c) st = issue_queries(s, s->cl[c]);
    if (st) {
      serve_fail(s, st);
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop; });
      break;
    }
    if (!progress) {
      // work is in flight: poll its events again shortly, or take new work
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait_for(lk, std::chrono::microseconds(20), [&] { return s->stop || !s->inbox.empty(); });
    }
  }
}

void server_free(Server* s) {
  lane_destroy(&s->alane);
  for (ClassLane& c : s->cl) {
    if (c.hdr) __atomic_store_n(&c.hdr->stop, 1, __ATOMIC_RELEASE);  // a running launch claims nothing more
    lane_destroy(&c.lane);  // waits for the class's stream
    if (c.kev) (void)hipEventDestroy(c.kev);
    if (c.host) (void)hipHostFree(c.host);
  }
  if (s->aev) (void)hipEventDestroy(s->aev);
  if (s->commit_ev) (void)hipEventDestroy(s->commit_ev);
  for (hipEvent_t ev : s->lev_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (Request* r : s->reqs) delete r;
  delete s;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_serve_start(tk_tree* t, const tk_serve_config* cfg) {
  if (!t) return TK_EINVAL;
  if (t->server) return fail(t, TK_EBUSY, "already serving");
  if (t->poisoned) return TK_EDEVICE;
  tk_serve_config c{};
  c.max_batch = 256;
  c.max_commit_blocks = 64;
  c.ws_budget_bytes = int64_t(1) << 30;
  c.max_queue = 1 << 20;
  if (cfg) {
    if (cfg->max_batch > 0) c.max_batch = cfg->max_batch;
    if (cfg->max_commit_blocks > 0) c.max_commit_blocks = cfg->max_commit_blocks;
    if (cfg->ws_budget_bytes > 0) c.ws_budget_bytes = cfg->ws_budget_bytes;
    if (cfg->max_queue > 0) c.max_queue = cfg->max_queue;
  }
  if (c.max_batch > (1 << 16) || c.max_commit_blocks > (1 << 16)) return fail(t, TK_EINVAL, "serve config too large");
  TK_HIP(t, hipStreamSynchronize(t->stream));
  Server* s = new Server();
  s->t = t;
  s->cfg = c;
  s->t0 = std::chrono::steady_clock::now();
  s->T_logical = t->T;
  s->Tb_issued = t->Tb;
  s->Tb_done = t->Tb;
  s->rows_staged = t->T % t->ell;
  s->stats.T_submitted = t->T;
  auto bail = [&](tk_status st) {
    server_free(s);
    return st;
  };
  hipError_t e = hipStreamCreateWithFlags(&s->alane.stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(fail_dev(t, e, "serve: append stream"));
  s->alane.own_stream = true;
  tk_status st = ensure(t, &s->alane.xbuf, int64_t(c.max_commit_blocks) * t->ell * t->slice_elems * 4, "serve staging");
  if (st) return bail(st);
  if (s->rows_staged > 0) {  // rows of a partial block appended before serving
    e = hipMemcpy(s->alane.xbuf.p, t->block_buf, size_t(s->rows_staged * t->slice_elems) * 4,
                  hipMemcpyDeviceToDevice);
    if (e != hipSuccess) return bail(fail_dev(t, e, "serve: staging"));
  }
  if ((e = hipEventCreateWithFlags(&s->aev, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&s->commit_ev, hipEventDisableTiming)) != hipSuccess)
    return bail(fail_dev(t, e, "serve: events"));
  for (int k = 0; k < MAXLEV; ++k) {
    if ((e = hipEventCreateWithFlags(&s->lev_ev[k], hipEventDisableTiming)) != hipSuccess)
      return bail(fail_dev(t, e, "serve: level events"));
    s->Tb_lvl[k] = t->Tb;
  }
  // size classes: small and medium narrow jobs, then wide ones
  const int cap = lds_cap(t);
  const int thr = t->tuning.wide_threshold < cap ? t->tuning.wide_threshold : cap;
  s->bounds[0] = thr < 32 ? thr : 32;
  s->bounds[1] = thr;
  s->bounds[2] = 1 << 30;
  for (int k = 0; k < kClasses; ++k) {
    ClassLane& cl = s->cl[k];
    cl.n_lds = k < kClasses - 1 ? s->bounds[k] : cap;
    const int hi = s->bounds[k];
    cl.threads = hi <= t->tuning.wide_threshold ? NT_STITCH : t->tuning.wide_threads;
    cl.ws_budget = c.ws_budget_bytes / kClasses;
    // dynamic LDS: every eigenproblem the class admits (the last class: up to
    // the LDS limit, for the vectors of eigenproblems beyond the cap)
    cl.lds_doubles = int(k < kClasses - 1 ? eig_doubles(cl.n_lds)
                                          : (t->lds_limit - int64_t(stitch_static_lds())) / 8);
    const int per_cu = stitch_blocks_per_cu(cl.threads, size_t(cl.lds_doubles) * 8);
    cl.grid = std::max(1, std::min(c.max_batch, std::max(1, per_cu) * t->n_cu / 2));
    cl.slots = int64_t(4) * c.max_batch;
    if ((e = hipStreamCreateWithFlags(&cl.lane.stream, hipStreamNonBlocking)) != hipSuccess)
      return bail(fail_dev(t, e, "serve: class stream"));
    cl.lane.own_stream = true;
    if ((e = hipEventCreateWithFlags(&cl.kev, hipEventDisableTiming)) != hipSuccess)
      return bail(fail_dev(t, e, "serve: class event"));
    if ((st = ensure(t, &cl.lane.ws[0], cl.ws_budget + 256, "serve workspace")) ||
        (st = ensure(t, &cl.lane.queue, 64, "serve ring head")))
      return bail(st);
    // ring: header | jobs | hits | statistics | completion words (host, mapped)
    const size_t o_jobs = 256;
    const size_t o_hits = o_jobs + size_t(align256(cl.slots * int64_t(sizeof(Job))));
    const size_t o_stats = o_hits + size_t(align256(cl.slots * MAXHITS * int64_t(sizeof(Hit))));
    const size_t o_done = o_stats + size_t(align256(cl.slots * STAT_COUNT * 8));
    const size_t bytes = o_done + size_t(cl.slots) * 8;
    if ((e = hipHostMalloc(&cl.host, bytes, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
      return bail(fail_dev(t, e, "serve: ring memory"));
    std::memset(cl.host, 0, bytes);
    void* dp = nullptr;
    if ((e = hipHostGetDevicePointer(&dp, cl.host, 0)) != hipSuccess)
      return bail(fail_dev(t, e, "serve: ring device address"));
    char* h = static_cast<char*>(cl.host);
    char* d = static_cast<char*>(dp);
    cl.hdr = reinterpret_cast<RingHdr*>(h);
    cl.hdr->slots = int32_t(cl.slots);
    cl.jobs = reinterpret_cast<Job*>(h + o_jobs);
    cl.hits = reinterpret_cast<Hit*>(h + o_hits);
    cl.stats = reinterpret_cast<double*>(h + o_stats);
    cl.done = reinterpret_cast<int64_t*>(h + o_done);
    cl.dhits = reinterpret_cast<Hit*>(d + o_hits);
    cl.dstats = reinterpret_cast<double*>(d + o_stats);
    cl.dring.hdr = reinterpret_cast<RingHdr*>(d);
    cl.dring.jobs = reinterpret_cast<const Job*>(d + o_jobs);
    cl.dring.done = reinterpret_cast<int64_t*>(d + o_done);
    cl.dring.head = reinterpret_cast<int64_t*>(cl.lane.queue.p);
    cl.dring.idle_ticks = kRingIdleTicks;
    cl.dring.life_ticks = kRingLifeTicks;
    cl.slot_req.assign(size_t(cl.slots), nullptr);
    if ((e = hipMemsetAsync(cl.lane.queue.p, 0, 64, cl.lane.stream)) != hipSuccess ||
        (e = hipStreamSynchronize(cl.lane.stream)) != hipSuccess)
      return bail(fail_dev(t, e, "serve: ring head"));
  }
  t->server = s;
  s->th = std::thread(engine, s);
  return TK_OK;
}

tk_status tk_serve_stop(tk_tree* t) {
  if (!t || !t->server) return TK_OK;
  Server* s = t->server;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  // committed blocks are on the append lane's stream: order the tree's
  // stream after them, and keep a partial block's rows for tk_append
  (void)hipStreamSynchronize(s->alane.stream);
  if (s->rows_staged > 0 && !s->failed)
    (void)hipMemcpy(t->block_buf, s->alane.xbuf.p, size_t(s->rows_staged * t->slice_elems) * 4,
                    hipMemcpyDeviceToDevice);
  t->T = s->T_logical;
  t->tail_rows = s->failed ? 0 : s->rows_staged;  // the incomplete block's rows, for tail queries
  t->prov_T = -1;
  const bool failed = s->failed;
  t->server = nullptr;
  server_free(s);
  return failed ? TK_EDEVICE : TK_OK;
}

tk_status tk_submit_query(tk_tree* t, int64_t ts, int64_t te, tk_result* res, uint64_t* ticket) {
  if (!t || !res || !ticket) return TK_EINVAL;
  Server* s = t->server;
  if (!s) return fail(t, TK_EINVAL, "not serving: call tk_serve_start");
  if (!res->core) return TK_EINVAL;
  for (int m = 0; m < t->p; ++m)
    if (!res->factor[m]) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) return TK_EDEVICE;
  if (s->outstanding >= s->cfg.max_queue) {
    s->stats.rejected += 1;
    return TK_EBUSY;
  }
  const int64_t Tb = s->T_logical / t->ell;
  if (!(ts >= 0 && ts < te && te <= Tb * t->ell)) return TK_ERANGE;
  Request* r = new Request();
  std::vector<Job> jobs;
  // planning only reads immutable tree fields (config, store layout)
  if (make_query_job(t, ts, te, Tb, res, true, jobs, r->hits) != TK_OK) {
    delete r;
    return TK_EINVAL;
  }
  r->job = jobs[0];
  r->job.hit0 = 0;
  StitchLayout lo;
  stitch_layout(t->view, r->hits.data(), r->job.s, r->job.rq, 1 << 30, &lo);
  r->need = eig_need(t, lo);
  r->cls = class_of(s, r->need);
  if (group_lds_doubles(s->cl[r->cls].n_lds, r->need) * 8 + int64_t(stitch_static_lds()) > t->lds_limit) {
    delete r;
    return TK_EINVAL;  // its eigenproblem's vectors do not fit in LDS
  }
  stitch_layout(t->view, r->hits.data(), r->job.s, r->job.rq, s->cl[r->cls].n_lds, &lo);
  r->job.ws_bytes = lo.total;
  if (lo.total > s->cl[r->cls].ws_budget) {
    delete r;
    s->stats.rejected += 1;
    return TK_ENOMEM;  // larger than the class's workspace budget
  }
  r->kind = 0;
  r->ts = ts;
  r->te = te;
  r->Tb = Tb;
  for (const Hit& h : r->hits) r->Tb_need = std::max(r->Tb_need, (h.index + 1) << h.level);
  r->res = res;
  r->ticket = uint64_t(s->reqs.size()) + 1;
  r->t_submit = now_us(s->t0);
  s->reqs.push_back(r);
  s->inbox.push_back(r);
  s->outstanding += 1;
  s->stats.queries += 1;
  *ticket = r->ticket;
  s->cv.notify_all();
  return TK_OK;
}

tk_status tk_submit_append(tk_tree* t, const float* slice, int on_device, uint64_t* ticket) {
  if (!t || !slice || !ticket) return TK_EINVAL;
  Server* s = t->server;
  if (!s) return fail(t, TK_EINVAL, "not serving: call tk_serve_start");
  Request* r = new Request();
  r->kind = 1;
  if (on_device) r->dev_slice = slice;
  else r->data.assign(slice, slice + t->slice_elems);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) {
    delete r;
    return TK_EDEVICE;
  }
  if (s->T_logical >= t->cap_blocks * t->ell) {
    delete r;
    return TK_ENOMEM;
  }
  if (s->outstanding >= s->cfg.max_queue) {
    delete r;
    s->stats.rejected += 1;
    return TK_EBUSY;
  }
  s->T_logical += 1;
  r->ticket = uint64_t(s->reqs.size()) + 1;
  r->t_submit = now_us(s->t0);
  s->reqs.push_back(r);
  s->inbox.push_back(r);
  s->outstanding += 1;
  s->stats.appends += 1;
  s->stats.T_submitted = s->T_logical;
  *ticket = r->ticket;
  s->cv.notify_all();
  return TK_OK;
}

tk_status tk_poll(tk_tree* t, uint64_t ticket, int32_t* done) {
  if (!t || !done) return TK_EINVAL;
  Server* s = t->server;
  if (!s) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket < 1 || ticket > s->reqs.size()) return TK_EINVAL;
  const Request* r = s->reqs[ticket - 1];
  *done = r->state >= REQ_DONE ? 1 : 0;
  return r->state == REQ_FAILED ? TK_EDEVICE : TK_OK;
}

tk_status tk_wait(tk_tree* t, uint64_t ticket) {
  if (!t) return TK_EINVAL;
  Server* s = t->server;
  if (!s) return TK_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket < 1 || ticket > s->reqs.size()) return TK_EINVAL;
  const Request* r = s->reqs[ticket - 1];
  s->done_cv.wait(lk, [&] { return r->state >= REQ_DONE; });
  return r->state == REQ_FAILED ? TK_EDEVICE : TK_OK;
}

tk_status tk_sync(tk_tree* t) {
  if (!t) return TK_EINVAL;
  Server* s = t->server;
  if (!s) {
    if (hipStreamSynchronize(t->stream) != hipSuccess) return TK_EDEVICE;
    return TK_OK;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  s->done_cv.wait(lk, [&] { return s->outstanding == 0; });
  return s->failed ? TK_EDEVICE : TK_OK;
}

tk_status tk_ticket_times(tk_tree* t, uint64_t ticket, double* submit_us, double* launch_us, double* done_us) {
  if (!t || !submit_us || !launch_us || !done_us) return TK_EINVAL;
  Server* s = t->server;
  if (!s) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket < 1 || ticket > s->reqs.size()) return TK_EINVAL;
  const Request* r = s->reqs[ticket - 1];
  *submit_us = r->t_submit;
  *launch_us = r->t_launch;
  *done_us = r->state >= REQ_DONE ? r->t_done : -1.0;
  return TK_OK;
}

tk_status tk_serve_stats_get(tk_tree* t, tk_serve_stats* out) {
  if (!t || !out) return TK_EINVAL;
  Server* s = t->server;
  if (!s) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->T_committed = s->Tb_done * t->ell;
  out->outstanding = s->outstanding;
  return TK_OK;
}

}  // extern "C"
