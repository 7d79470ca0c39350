// Prepared query batches and the launch autotuner.
//
// A prepared batch plans a fixed list of range queries once (Recall for the
// workspace sizes, LDS bins, heaviest-first order), uploads the job
// descriptors, and captures its launches in a HIP graph: per LDS bin, the
// trim pass over the long partial hits' rows, then one fused stitch kernel
// running Recall, the partial-hit trims and the Stitch of its queries, the
// bins forked onto their own streams and joined.
// tk_batch_run replays the graph on the tree's stream.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tk_host.hpp"
#include "tk_tune_search.hpp"

using namespace tk;

struct tk_batch {
  tk_tree* t = nullptr;
  int32_t n = 0;
  tk_result* res = nullptr;
  std::vector<Job> qjobs;  // in the caller's order (ranks, hit counts)
  Plan plan;
  DevBuf hits, stats, queue, ws[kMaxGroups], jobs[kMaxGroups], trims[kMaxGroups];
  int64_t n_trims[kMaxGroups] = {};  // chunks of the trim pass per group
  hipStream_t cap_stream = nullptr;
  hipStream_t gstream[kMaxGroups] = {};
  hipEvent_t gev[kMaxGroups] = {};
  hipEvent_t fork_ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool ran = false;
  std::vector<double> hstats;
};

namespace {

void batch_free(tk_batch* b) {
  if (!b) return;
  tk_tree* t = b->t;
  if (t && t->stream) (void)hipStreamSynchronize(t->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  release(&b->hits);
  release(&b->stats);
  release(&b->queue);
  for (int g = 0; g < kMaxGroups; ++g) {
    release(&b->ws[g]);
    release(&b->jobs[g]);
    release(&b->trims[g]);
    if (b->gstream[g]) (void)hipStreamDestroy(b->gstream[g]);
    if (b->gev[g]) (void)hipEventDestroy(b->gev[g]);
  }
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete b;
}

// Enqueue the batch's kernels on `stream` (captured or direct): every group
// on its own stream, forked from and joined back to `stream`.
tk_status issue(tk_batch* b, hipStream_t stream) {
  tk_tree* t = b->t;
  StitchArgs base = stitch_args(t, t->q_max_iter, t->q_tol);
  base.basis_pct = b->plan.basis_pct;
  base.hits = reinterpret_cast<Hit*>(b->hits.p);
  const bool fork = b->plan.groups.size() > 1;
  bool used[kForkStreams] = {false, false, false, false};
  if (fork) TK_HIP(t, hipEventRecord(b->fork_ev, stream));
  for (const Group& gr : b->plan.groups) {
    const int g = gr.bin;
    hipStream_t s = fork ? b->gstream[gr.slot] : stream;
    if (fork && !used[gr.slot]) TK_HIP(t, hipStreamWaitEvent(s, b->fork_ev, 0));
    if (fork) used[gr.slot] = true;
    const size_t lds_bytes = size_t(gr.lds_doubles) * 8;
    StitchArgs a = base;
    a.jobs = reinterpret_cast<const Job*>(b->jobs[g].p);
    a.ws = b->ws[g].p;
    a.n_jobs = int(gr.jobs.size());
    a.n_lds = gr.n_lds;
    a.lds_doubles = gr.lds_doubles;
    int grid = a.n_jobs;
    a.queue = nullptr;
    if (t->tuning.persistent) {
      const int64_t resident = int64_t(stitch_blocks_per_cu(gr.threads, lds_bytes)) * t->n_cu;
      if (resident < grid) grid = int(resident);
      a.queue = reinterpret_cast<int*>(b->queue.p) + g;
      TK_HIP(t, launch_reset_queue(a.queue, 1, s));
    }
    if (b->n_trims[g] > 0)  // the trim pass first: row Grams of the long partial hits
      TK_HIP(t, launch_trim(reinterpret_cast<const TrimChunk*>(b->trims[g].p), b->n_trims[g], s));
    TK_HIP(t, launch_stitch(a, grid, lds_bytes, gr.threads, s));
  }
  for (int sl = 0; sl < kForkStreams && fork; ++sl) {
    if (!used[sl]) continue;
    TK_HIP(t, hipEventRecord(b->gev[sl], b->gstream[sl]));
    TK_HIP(t, hipStreamWaitEvent(stream, b->gev[sl], 0));
  }
  return TK_OK;
}

}  // namespace

extern "C" {

tk_status tk_batch_create(tk_tree* t, int32_t n, const int64_t* ts, const int64_t* te, tk_result* res,
                          tk_batch** out) {
  if (!t || !out || n < 1 || !ts || !te || !res) return fail(t, TK_EINVAL, "bad argument");
  *out = nullptr;
  if (t->server) return fail(t, TK_EBUSY, "the tree is serving; stop the server first");
  if (t->poisoned) return TK_EDEVICE;
  tk_batch* b = new tk_batch();
  b->t = t;
  b->n = n;
  b->res = res;
  std::vector<Hit> hits;
  for (int32_t i = 0; i < n; ++i) {
    tk_status st = make_query_job(t, ts[i], te[i], t->Tb, &res[i], true, b->qjobs, hits);
    if (st) {
      batch_free(b);
      return st;
    }
  }
  auto bail = [&](tk_status st) {
    batch_free(b);
    return st;
  };
  tk_status st = ensure(t, &b->stats, int64_t(n) * STAT_COUNT * 8, "stats");
  if (st) return bail(st);
  double* dstats = reinterpret_cast<double*>(b->stats.p);
  std::vector<Job> jobs = b->qjobs;
  for (int32_t i = 0; i < n; ++i) jobs[i].stats = dstats + STAT_COUNT * int64_t(i);
  st = plan_stitch(t, jobs, hits, &b->plan, true);
  if (st) return bail(st);
  // the kernels run Recall themselves and write the hits; their slots start
  // zeroed (queries on host-planned hits, kind 2, get the plan's)
  st = ensure(t, &b->hits, int64_t(hits.size() * sizeof(Hit)) + 64, "hits");
  if (st) return bail(st);
  TK_HIP(t, hipMemset(b->hits.p, 0, size_t(b->hits.cap)));
  {
    std::vector<Hit> planned(hits.size(), Hit{});
    bool any = false;
    for (const Job& jb : b->qjobs)
      if (jb.kind == 2) {
        for (int k = 0; k < jb.s; ++k) planned[size_t(jb.hit0 + k)] = hits[size_t(jb.hit0 + k)];
        any = true;
      }
    if (any)
      TK_HIP(t, hipMemcpy(b->hits.p, planned.data(), planned.size() * sizeof(Hit), hipMemcpyHostToDevice));
  }
  st = ensure(t, &b->queue, kMaxGroups * 64, "queue");
  if (st) return bail(st);
  TK_HIP(t, hipMemset(b->queue.p, 0, size_t(b->queue.cap)));
  TK_HIP(t, hipMemset(b->stats.p, 0, size_t(b->stats.cap)));
  for (const Group& gr : b->plan.groups) {
    if (int64_t(gr.jobs.size()) > (int64_t(1) << 24)) return bail(fail(t, TK_EINVAL, "batch too large"));
    st = ensure(t, &b->ws[gr.bin], gr.ws_total + 256, "batch workspace");
    if (st) return bail(st);
    st = ensure(t, &b->jobs[gr.bin], int64_t(gr.jobs.size() * sizeof(Job)), "batch jobs");
    if (st) return bail(st);
    TK_HIP(t, hipMemcpy(b->jobs[gr.bin].p, gr.jobs.data(), gr.jobs.size() * sizeof(Job), hipMemcpyHostToDevice));
    std::vector<TrimChunk> trims;
    trim_chunks_of(t, b->plan, gr, 0, int64_t(gr.jobs.size()), b->ws[gr.bin].p, trims);
    b->n_trims[gr.bin] = int64_t(trims.size());
    if (!trims.empty()) {
      st = ensure(t, &b->trims[gr.bin], int64_t(trims.size() * sizeof(TrimChunk)), "batch trim chunks");
      if (st) return bail(st);
      TK_HIP(t, hipMemcpy(b->trims[gr.bin].p, trims.data(), trims.size() * sizeof(TrimChunk), hipMemcpyHostToDevice));
    }
    if (!b->gstream[gr.slot]) {
      TK_HIP(t, hipStreamCreateWithFlags(&b->gstream[gr.slot], hipStreamNonBlocking));
      TK_HIP(t, hipEventCreateWithFlags(&b->gev[gr.slot], hipEventDisableTiming));
    }
  }
  TK_HIP(t, hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  TK_HIP(t, hipEventCreate(&b->ev0));
  TK_HIP(t, hipEventCreate(&b->ev1));
  if (t->tuning.graph) {
    TK_HIP(t, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    TK_HIP(t, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    st = issue(b, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return bail(st);
    }
    if (e != hipSuccess) return bail(fail_dev(t, e, "hipStreamEndCapture"));
    b->graph = g;
    TK_HIP(t, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  *out = b;
  return TK_OK;
}

tk_status tk_batch_run(tk_batch* b) {
  if (!b) return TK_EINVAL;
  tk_tree* t = b->t;
  if (t->server) return fail(t, TK_EBUSY, "the tree is serving; stop the server first");
  if (t->poisoned) return TK_EDEVICE;
  TK_HIP(t, hipEventRecord(b->ev0, t->stream));
  if (b->exec) {
    TK_HIP(t, hipGraphLaunch(b->exec, t->stream));
  } else {
    tk_status st = issue(b, t->stream);
    if (st) return st;
  }
  TK_HIP(t, hipEventRecord(b->ev1, t->stream));
  b->ran = true;
  return TK_OK;
}

tk_status tk_batch_wait(tk_batch* b) {
  if (!b) return TK_EINVAL;
  tk_tree* t = b->t;
  if (!b->ran) return fail(t, TK_EINVAL, "batch has not run");
  TK_HIP(t, hipEventSynchronize(b->ev1));
  b->hstats.assign(size_t(b->n) * STAT_COUNT, 0.0);
  TK_HIP(t, hipMemcpy(b->hstats.data(), b->stats.p, b->hstats.size() * 8, hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < b->n; ++i) {
    const double* s = b->hstats.data() + STAT_COUNT * size_t(i);
    if (s[STAT_STATUS] != 0.0)
      return fail(t, TK_EDEVICE, job_status_msg(s[STAT_STATUS]));
    tk_result& r = b->res[i];
    for (int m = 0; m < TK_MAX_MODES; ++m) r.ranks_eff[m] = m < t->p ? b->qjobs[i].rq[m] : 0;
    r.fit = s[STAT_FIT];
    r.err_model = s[STAT_ERR];
    r.norm_ytilde = s[STAT_NORM];
    r.sweeps = int32_t(s[STAT_SWEEPS]);
    r.converged = int32_t(s[STAT_CONV]);
    r.n_hits = b->qjobs[i].s;
  }
  return TK_OK;
}

tk_status tk_batch_kernel_ms(const tk_batch* b, double* ms) {
  if (!b || !ms || !b->ran) return TK_EINVAL;
  float f = 0.f;
  if (hipEventSynchronize(b->ev1) != hipSuccess) return TK_EDEVICE;
  if (hipEventElapsedTime(&f, b->ev0, b->ev1) != hipSuccess) return TK_EDEVICE;
  *ms = double(f);
  return TK_OK;
}

tk_status tk_batch_profile(const tk_batch* b, int32_t i, double* phase_us) {
  if (!b || !phase_us || i < 0 || i >= b->n) return TK_EINVAL;
  if (b->hstats.size() != size_t(b->n) * STAT_COUNT) return TK_EINVAL;
  for (int k = 0; k < PROFILE_COUNT; ++k)
    phase_us[k] = b->hstats[size_t(i) * STAT_COUNT + STAT_PHASE + k] *
                  (k == STAT_NPHASE + 4 || k == STAT_NPHASE + 5 ? 0.01 : 1.0);
  return TK_OK;
}

tk_status tk_batch_hits(const tk_batch* b, int32_t i, tk_hit* out, int32_t cap, int32_t* n) {
  if (!b || !n || i < 0 || i >= b->n || (cap > 0 && !out)) return TK_EINVAL;
  tk_tree* t = b->t;
  const Job& jb = b->qjobs[i];
  std::vector<Hit> h(static_cast<size_t>(jb.s));
  if (hipMemcpy(h.data(), b->hits.p + size_t(jb.hit0) * sizeof(Hit), h.size() * sizeof(Hit),
                hipMemcpyDeviceToHost) != hipSuccess)
    return TK_EDEVICE;
  *n = jb.s;
  for (int k = 0; k < jb.s && k < cap; ++k) {
    const int64_t sig = (h[k].index << h[k].level) * t->ell;
    out[k].level = h[k].level;
    out[k].index = h[k].index;
    out[k].partial = h[k].partial;
    out[k].node_id = node_id(h[k].level, h[k].index);
    out[k].sigma = sig;
    out[k].tau = sig + (t->ell << h[k].level);
    out[k].lo = sig + h[k].a;
    out[k].hi = sig + h[k].a + h[k].l;
  }
  return TK_OK;
}

void tk_batch_destroy(tk_batch* b) { batch_free(b); }

tk_status tk_set_autotune_limits(tk_tree* t, double budget_s, double cap, int32_t progress) {
  if (!t || !(budget_s >= 0.0) || !(cap >= 0.0)) return fail(t, TK_EINVAL, "bad autotune limits");
  t->tune_limits.budget_s = budget_s;
  t->tune_limits.cap = cap;
  t->tune_limits.progress = progress ? 1 : 0;
  return TK_OK;
}

tk_status tk_autotune(tk_tree* t, int32_t n, const int64_t* ts, const int64_t* te, int32_t reps, tk_tuning* best,
                      double* best_ms) {
  if (!t || n < 1 || !ts || !te || reps < 1) return fail(t, TK_EINVAL, "bad argument");
  if (t->server) return fail(t, TK_EBUSY, "the tree is serving; stop the server first");
  if (t->poisoned) return TK_EDEVICE;
  // scratch outputs for the sample
  int64_t total = 0;
  std::vector<int64_t> off(static_cast<size_t>(n) * (t->p + 1));
  for (int32_t i = 0; i < n; ++i) {
    if (!(ts[i] >= 0 && ts[i] < te[i] && te[i] <= t->Tb * t->ell)) return fail(t, TK_ERANGE, "query range");
    int32_t r[MAXP];
    query_ranks(t, te[i] - ts[i], r);
    int64_t ce = 1;
    for (int m = 0; m < t->p; ++m) ce *= r[m];
    off[size_t(i) * (t->p + 1)] = total;
    total += ce;
    off[size_t(i) * (t->p + 1) + 1] = total;
    total += (te[i] - ts[i]) * r[0];
    for (int m = 1; m < t->p; ++m) {
      off[size_t(i) * (t->p + 1) + 1 + m] = total;
      total += t->view.D[m] * r[m];
    }
  }
  DevBuf outbuf;
  tk_status st = ensure(t, &outbuf, total * 4 + 256, "autotune outputs");
  if (st) return st;
  float* base = reinterpret_cast<float*>(outbuf.p);
  std::vector<tk_result> res(static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i) {
    std::memset(&res[i], 0, sizeof(tk_result));
    res[i].core = base + off[size_t(i) * (t->p + 1)];
    for (int m = 0; m < t->p; ++m) res[i].factor[m] = base + off[size_t(i) * (t->p + 1) + 1 + m];
  }
  const Tuning saved = t->tuning;
  Tuning bestt = saved;
  double bms = 1e300;
  const auto clock0 = std::chrono::steady_clock::now();
  auto now_s = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - clock0).count(); };
  TuneSearch search(t->tune_limits, 0.0);
  bool abandoned = false;
  // time the tree's current tuning on the sample: one warm-up execution,
  // then nrep timed ones unless the warm-up alone rules the candidate out;
  // false on an error (st set)
  std::vector<std::pair<double, Tuning>> timed;
  auto time_it = [&](int nrep, double* out_ms) {
    tk_batch* b = nullptr;
    st = tk_batch_create(t, n, ts, te, res.data(), &b);
    double sum = 0.0;
    int done = 0;
    abandoned = false;
    for (int r = 0; r <= nrep && st == TK_OK; ++r) {
      st = tk_batch_run(b);
      if (st == TK_OK) st = tk_batch_wait(b);
      double ms = 0.0;
      if (st == TK_OK) st = tk_batch_kernel_ms(b, &ms);
      if (st != TK_OK) break;
      if (r == 0 && !search.worth_timing(ms)) {
        abandoned = true;
        sum = ms;
        done = 1;
        break;
      }
      if (r > 0) {  // the first run warms up
        sum += ms;
        ++done;
      }
    }
    tk_batch_destroy(b);
    *out_ms = done ? sum / done : 0.0;
    return st == TK_OK;
  };
  auto describe = [&](char* buf, size_t len) {
    const Tuning& u = t->tuning;
    std::snprintf(buf, len,
                  "wide_threshold %d wide_threads %d persistent %d coarse %d lds_n %d basis_pct %d rest_threads %d "
                  "wide_core %d",
                  u.wide_threshold, u.wide_threads, u.persistent, u.coarse, u.lds_n, u.basis_pct, u.rest_threads,
                  u.wide_core);
  };
  // false on an error or once the time budget is spent (ok then stays true)
  bool budget_left = true;
  auto trial = [&]() {
    if (!search.open(now_s())) {
      budget_left = false;
      return false;
    }
    double ms = 0.0;
    if (!time_it(reps, &ms)) return false;
    char what[192];
    describe(what, sizeof(what));
    search.record(ms, abandoned, what, now_s());
    if (abandoned) return true;
    timed.push_back({ms, t->tuning});
    if (ms < bms) {
      bms = ms;
      bestt = t->tuning;
    }
    return true;
  };
  const int thr[] = {32, 48, 64, 96};
  const int wth[] = {128, 256};
  const int ldsn[] = {32, 48, 64, 96, 0};
  bool ok = true;
  for (int th : thr)
    for (int wt : wth)
      for (int ln : ldsn)
        for (int pc = 0; pc < 4 && ok && budget_left; ++pc) {
          if (ln != 0 && ln < th) continue;
          t->tuning = saved;
          t->tuning.wide_threshold = th;
          t->tuning.wide_threads = wt;
          t->tuning.lds_n = ln;
          t->tuning.persistent = pc & 1;
          t->tuning.coarse = pc >> 1;
          t->tuning.basis_pct = 75;
          t->tuning.rest_threads = 0;
          t->tuning.wide_core = 0;
          ok = trial() || (st == TK_OK && !budget_left);
        }
  const int bpct[] = {60, 90, 100};
  Tuning from = bestt;
  for (int bp : bpct) {
    if (!ok || !budget_left) break;
    t->tuning = from;
    t->tuning.basis_pct = bp;
    ok = trial() || (st == TK_OK && !budget_left);
  }
  const int rth[] = {128, 256};
  from = bestt;
  for (int rt : rth) {
    if (!ok || !budget_left || rt == from.wide_threads) continue;
    t->tuning = from;
    t->tuning.rest_threads = rt;
    ok = trial() || (st == TK_OK && !budget_left);
  }
  const int wcs[] = {2048, 8192};
  from = bestt;
  for (int wc : wcs) {
    if (!ok || !budget_left) break;
    t->tuning = from;
    t->tuning.wide_core = wc;
    ok = trial() || (st == TK_OK && !budget_left);
  }
  // single timings pick the luckiest point: the eight fastest are timed
  // again, three times as long, and the best mean wins
  // (skipped once the budget is spent)
  if (ok && budget_left && timed.size() > 1) {
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<double, Tuning>& x, const std::pair<double, Tuning>& y) {
                       return x.first < y.first;
                     });
    const double single_best = bms;
    double rbest = 1e300;
    Tuning rt = bestt;
    bool complete = true;
    for (size_t c = 0; c < timed.size() && c < 8 && ok; ++c) {
      if (!search.open(now_s())) {
        complete = false;
        break;
      }
      t->tuning = timed[c].second;
      double ms = 0.0;
      ok = time_it(3 * reps, &ms);
      if (ok && !abandoned && ms < rbest) {
        rbest = ms;
        rt = timed[c].second;
      }
    }
    // keep the re-timed winner only when every re-timing ran
    if (ok && complete && rbest < 1e300) {
      bms = rbest;
      bestt = rt;
    } else {
      bms = single_best;
    }
  }
  if (t->tune_limits.progress)
    std::fprintf(stderr, "[tk_autotune] %d candidates (%d abandoned after warm-up) in %.1f s%s; best %.3f ms\n",
                 search.count(), search.abandoned(), now_s(), budget_left ? "" : " (time budget spent)", bms);
  if (!ok) {
    t->tuning = saved;
    release(&outbuf);
    return st;
  }
  t->tuning = bestt;
  release(&outbuf);
  if (best) {
    best->wide_threshold = bestt.wide_threshold;
    best->wide_threads = bestt.wide_threads;
    best->persistent = bestt.persistent;
    best->graph = bestt.graph;
    best->coarse = bestt.coarse;
    best->lds_n = bestt.lds_n;
    best->basis_pct = bestt.basis_pct;
    best->rest_threads = bestt.rest_threads;
    best->wide_core = bestt.wide_core;
  }
  if (best_ms) *best_ms = bms;
  return TK_OK;
}

}  // extern "C"
