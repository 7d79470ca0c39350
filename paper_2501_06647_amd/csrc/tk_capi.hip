// C ABI of the TUCKET engine: tree object, node store, append/build
// scheduling and query launches.  Integer work (which nodes, where they live)
// happens here on the host; every floating-point step runs in the kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tk_host.hpp"

using tk::Hit;
using tk::Job;
using tk::LeafJob;
using tk::StoreView;

namespace {
thread_local std::string g_create_error;
}  // namespace

namespace tk {

// Device scratch of tk_query_noalloc: a file-scope array that every device
// loading the library holds until the process ends.  Host code never uses
// its name as an address (on the host it names a stand-in, not device
// memory): tk_create looks up its address on the tree's device once per
// device (hipGetSymbolAddress, with that device current), and the entry
// point passes that address to the kernels like any other buffer.
constexpr int64_t kNoAllocScratchBytes = int64_t(32) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The scratch's address on device dev (the current device); nullptr with
// *err set if it cannot be found.
char* noalloc_scratch(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace tk

namespace tk {

void set_error(tk_tree* t, const std::string& msg) {
  std::lock_guard<std::mutex> lk(t->err_mu);
  t->err = msg;
}

tk_status fail(tk_tree* t, tk_status st, const std::string& msg) {
  if (t) set_error(t, msg);
  else g_create_error = msg;
  return st;
}

std::string job_status_msg(double status) {
  return "stitch kernel: job status " + std::to_string(int(status)) +
         " (1 device Recall, 2 workspace, 3 LDS or kernel modes) disagrees with the host plan";
}

tk_status fail_dev(tk_tree* t, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (t) {
    t->poisoned = true;
    set_error(t, m);
  } else {
    g_create_error = m;
  }
  return TK_EDEVICE;
}

tk_status ensure(tk_tree* t, DevBuf* b, int64_t need, const char* what) {
  if (need <= b->cap) return TK_OK;
  if (b->fixed) return fail(t, TK_ENOMEM, std::string(what) + ": exceeds the fixed scratch");
  if (b->p) {
    TK_HIP(t, hipDeviceSynchronize());  // the buffer may be in use on any of the tree's streams
    TK_HIP(t, hipFree(b->p));
    b->p = nullptr;
    b->cap = 0;
  }
  const int64_t sz = need + need / 4 + 4096;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, size_t(sz));
  if (e != hipSuccess) return fail_dev(t, e, what);
  b->p = static_cast<char*>(p);
  b->cap = sz;
  return TK_OK;
}

void release(DevBuf* b) {
  if (b->fixed) return;
  if (b->p) (void)hipFree(b->p);
  b->p = nullptr;
  b->cap = 0;
}

void lane_destroy(Lane* l) {
  if (l->stream) (void)hipStreamSynchronize(l->stream);
  for (int g = 0; g < kMaxGroups; ++g)
    if (l->gstream[g]) (void)hipStreamSynchronize(l->gstream[g]);
  release(&l->hits);
  release(&l->stats);
  release(&l->queue);
  release(&l->leaf_ws);
  release(&l->leaf_jobs);
  release(&l->xbuf);
  for (DevBuf& b : l->sx) release(&b);
  for (int g = 0; g < kMaxGroups; ++g) {
    release(&l->ws[g]);
    release(&l->jobs[g]);
    release(&l->trims[g]);
    if (l->gstream[g]) (void)hipStreamDestroy(l->gstream[g]);
    if (l->gev[g]) (void)hipEventDestroy(l->gev[g]);
    l->gstream[g] = nullptr;
    l->gev[g] = nullptr;
  }
  if (l->fork_ev) (void)hipEventDestroy(l->fork_ev);
  l->fork_ev = nullptr;
  if (l->own_stream && l->stream) (void)hipStreamDestroy(l->stream);
  l->stream = nullptr;
}

int eig_need(const tk_tree* t, const StitchLayout& lo) { return stitch_eig_need(lo, t->view, t->tuning.basis_pct); }

int query_hits(const tk_tree* t, int64_t ts, int64_t te, int64_t Tb, Hit* out, int cap) {
  if (t->q_level < 0) return recall(ts, te, Tb, t->ell, t->cfg.theta_num, t->cfg.theta_den, out, cap);
  return fixed_block_hits(ts, te, Tb, t->ell, t->q_level, t->cfg.theta_num, t->cfg.theta_den, out, cap);
}

void query_ranks(const tk_tree* t, int64_t len, int32_t* out) {
  int32_t req[MAXP];
  for (int n = 0; n < t->p; ++n) req[n] = t->q_ranks[n] > 0 ? t->q_ranks[n] : t->cfg.ranks[n];
  effective_ranks(t->p, len, t->view.D, req, out);
}

int64_t group_lds_doubles(int n_lds, int need) {
  return std::max(eig_doubles(n_lds), need > n_lds ? eig_vec_doubles(need) : int64_t(0));
}

int lds_cap(const tk_tree* t) {
  int cap = 128;
  while (cap > 8 && int64_t(eig_doubles(cap)) * 8 > t->lds_limit - int64_t(stitch_static_lds())) cap -= 8;
  if (t->tuning.lds_n > 0 && t->tuning.lds_n < cap) cap = t->tuning.lds_n;
  return cap;
}

StitchArgs stitch_args(tk_tree* t, int max_iter, double tol) {
  StitchArgs a{};
  a.st = t->dview;
  a.p = t->p;
  a.max_iter = max_iter;
  a.tol = tol;
  a.merge_max_iter = t->cfg.max_iter;
  a.merge_tol = t->cfg.tol;
  a.basis_pct = t->tuning.basis_pct;
  a.bf16 = t->q_prec == TK_BF16 ? 1 : 0;
  a.merge_bf16 = t->cfg.prec == TK_BF16 ? 1 : 0;
  a.theta_num = t->cfg.theta_num;
  a.theta_den = t->cfg.theta_den;
  return a;
}

int plan_query_hits(const tk_tree* t, int64_t ts, int64_t te, int64_t Tb, bool tail_ok, Hit* out, int cap,
                    bool* tail) {
  const int64_t Tc = Tb * t->ell;
  // the incomplete block is reachable when its slices were all appended here
  // (not after a restore or a serving session)
  const int64_t end = tail_ok && Tb == t->Tb && t->tail_rows == t->T - Tc ? t->T : Tc;
  *tail = false;
  if (!(ts >= 0 && ts < te && te <= end)) return -1;
  const int64_t tec = te < Tc ? te : Tc;
  int n = ts < tec ? query_hits(t, ts, tec, Tb, out, cap) : 0;
  if (te > Tc) {
    const int64_t lo = ts > Tc ? ts : Tc;
    if (n < cap) out[n] = Hit{0, 1, Tb, lo - Tc, te - lo};
    ++n;
    *tail = true;
  }
  return n;
}

tk_status make_query_job(tk_tree* t, int64_t ts, int64_t te, int64_t Tb, const tk_result* res, bool check_outputs,
                         std::vector<Job>& jobs, std::vector<Hit>& hits, bool tail_ok) {
  Hit buf[MAXHITS];
  bool tail = false;
  const int n = plan_query_hits(t, ts, te, Tb, tail_ok, buf, MAXHITS, &tail);
  if (n < 0) return fail(t, TK_ERANGE, "query range outside [0, T_c) or empty");
  if (n < 1 || n > MAXHITS) return fail(t, TK_EINVAL, "hit set too large");
  Job jb{};
  jb.kind = t->q_level < 0 && !tail ? 0 : 2;
  jb.s = n;
  jb.hit0 = int32_t(hits.size());
  jb.L = te - ts;
  jb.ts = ts;
  jb.Tb = Tb;
  query_ranks(t, te - ts, jb.rq);
  if (check_outputs) {
    if (!res || !res->core) return fail(t, TK_EINVAL, "null core buffer");
    for (int m = 0; m < t->p; ++m)
      if (!res->factor[m]) return fail(t, TK_EINVAL, "null factor buffer");
  }
  if (res) {
    jb.out_core = res->core;
    for (int m = 0; m < t->p; ++m) jb.out_fac[m] = res->factor[m];
  }
  for (int i = 0; i < n; ++i) hits.push_back(buf[i]);
  jobs.push_back(jb);
  return TK_OK;
}

void make_merge_job(tk_tree* t, int k, int64_t j, std::vector<Job>& jobs, std::vector<Hit>& hits) {
  const StoreView& v = t->view;
  Job jb{};
  jb.kind = 1;
  jb.s = 2;
  jb.hit0 = int32_t(hits.size());
  jb.L = t->ell << k;
  jb.ts = (j << k) * t->ell;
  jb.Tb = (j + 1) << k;
  for (int n = 0; n < t->p; ++n) jb.rq[n] = v.rk[k][n];
  jb.out_core = v.core[k] + j * v.core_elems[k];
  for (int n = 1; n < t->p; ++n) jb.out_fac[n] = v.fac[k][n] + j * fac_elems(v, k, n);
  jb.out_fac[0] = v.plane[k] + (j << k) * t->ell * v.rk[k][0];
  jb.stats = nullptr;
  const int64_t half = t->ell << (k - 1);
  Hit h0{k - 1, 0, 2 * j, 0, half};
  Hit h1{k - 1, 0, 2 * j + 1, 0, half};
  hits.push_back(h0);
  hits.push_back(h1);
  jobs.push_back(jb);
}

tk_status plan_stitch(tk_tree* t, std::vector<Job>& jobs, std::vector<Hit>& hits, Plan* plan, bool pretrim) {
  plan->groups.clear();
  plan->n_jobs = int64_t(jobs.size());
  plan->basis_pct = t->tuning.basis_pct;
  const int cap = lds_cap(t);
  const Tuning& tu = t->tuning;
  // bin bounds: fixed sizes plus the wide threshold, capped by the LDS limit;
  // the last bin takes everything above (eigenproblems beyond cap run in HBM)
  std::vector<int> bounds = tu.coarse ? std::vector<int>{32, 96} : std::vector<int>{24, 32, 48, 64, 96};
  if (tu.wide_threshold < cap) bounds.push_back(tu.wide_threshold);
  for (int& b : bounds) b = b < cap ? b : cap;
  std::sort(bounds.begin(), bounds.end());
  bounds.erase(std::unique(bounds.begin(), bounds.end()), bounds.end());
  while (int(bounds.size()) > kMaxGroups - 1) bounds.erase(bounds.begin());
  const int nb = int(bounds.size()) + 1;
  std::vector<Group> g(static_cast<size_t>(nb));
  for (int b = 0; b < nb; ++b) {
    g[b].bin = b;
    g[b].n_lds = b < nb - 1 ? bounds[b] : cap;
    const int hi = b < nb - 1 ? bounds[b] : (1 << 30);
    const int wide = b == nb - 1 && tu.rest_threads ? tu.rest_threads : tu.wide_threads;
    g[b].threads = hi <= tu.wide_threshold ? NT_STITCH : wide;
  }
  std::vector<int> maxneed(static_cast<size_t>(nb), 0);
  for (Job& jb : jobs) {
    StitchLayout lo;
    stitch_layout(t->view, hits.data() + jb.hit0, jb.s, jb.rq, 1 << 30, &lo);
    int need = eig_need(t, lo);
    if (need > EIG_MAXK_HOST) return fail(t, TK_EINVAL, "query needs an eigenproblem above 1024");
    if (tu.wide_core > 0 && need <= tu.wide_threshold) {  // small eigenproblems, large contractions
      int64_t core = 1;
      for (int m = 0; m < t->p; ++m) core *= jb.rq[m];
      if (core > tu.wide_core) need = tu.wide_threshold + 1;
    }
    int b = nb - 1;
    for (int k = 0; k < nb - 1; ++k)
      if (need <= bounds[k]) {
        b = k;
        break;
      }
    g[b].jobs.push_back(jb);
    maxneed[b] = std::max(maxneed[b], need);
  }
  for (Group& gr : g) {
    if (gr.jobs.empty()) continue;
    const int64_t ld = group_lds_doubles(gr.n_lds, maxneed[gr.bin]);
    if (ld * 8 + int64_t(stitch_static_lds()) > t->lds_limit)
      return fail(t, TK_EINVAL, "eigenproblem vectors exceed the LDS limit");
    gr.lds_doubles = int(ld);
    std::stable_sort(gr.jobs.begin(), gr.jobs.end(), [](const Job& a, const Job& b) {
      return a.s * a.L > b.s * b.L;  // longer ranges with more hits take longer
    });
    int64_t off = 0;
    for (Job& jb : gr.jobs) {
      jb.pretrim = 0;
      if (pretrim && jb.kind != 1) {
        int64_t rows = 0;
        for (int i = 0; i < jb.s; ++i)
          if (hits[size_t(jb.hit0 + i)].partial) rows += hits[size_t(jb.hit0 + i)].l;
        jb.pretrim = rows >= kPretrimRows ? 1 : 0;
      }
      StitchLayout lo;
      stitch_layout(t->view, hits.data() + jb.hit0, jb.s, jb.rq, gr.n_lds, &lo, jb.pretrim);
      jb.ws_off = off;
      jb.ws_bytes = lo.total;
      off += lo.total;
    }
    gr.ws_total = off;
    plan->groups.push_back(std::move(gr));
  }
  // heaviest group first; groups are dealt to the fork streams in that order
  std::stable_sort(plan->groups.begin(), plan->groups.end(), [](const Group& a, const Group& b) {
    return a.jobs[0].s * a.jobs[0].L > b.jobs[0].s * b.jobs[0].L;
  });
  for (size_t i = 0; i < plan->groups.size(); ++i) plan->groups[i].slot = int(i % kForkStreams);
  plan->hits = hits;
  return TK_OK;
}

void trim_chunks_of(const tk_tree* t, const Plan& plan, const Group& gr, int64_t i0, int64_t i1, char* ws_base,
                    std::vector<TrimChunk>& out) {
  const StoreView& v = t->view;
  const int64_t base_off = gr.jobs[size_t(i0)].ws_off;
  for (int64_t j = i0; j < i1; ++j) {
    const Job& jb = gr.jobs[size_t(j)];
    if (!jb.pretrim) continue;
    const Hit* hs = plan.hits.data() + jb.hit0;
    StitchLayout lo;
    stitch_layout(v, hs, jb.s, jb.rq, gr.n_lds, &lo, 1);
    double* tg = reinterpret_cast<double*>(ws_base + (jb.ws_off - base_off) + lo.TG);
    for (int i = 0; i < jb.s; ++i) {
      const Hit& h = hs[i];
      if (!h.partial) continue;
      const int k = v.rk[h.level][0];
      const float* V = v.plane[h.level] + ((h.index << h.level) * v.ell + h.a) * k;
      for (int64_t c = 0; c < trim_chunks(h.l); ++c) {
        const int64_t r0 = c * TRIM_CHUNK;
        TrimChunk ch{};
        ch.V = V + r0 * k;
        ch.rows = std::min<int64_t>(TRIM_CHUNK, h.l - r0);
        ch.out = tg;
        ch.k = k;
        out.push_back(ch);
        tg += int64_t(k) * k;
      }
    }
  }
}

namespace {

// Launch one group (chunked by workspace size) on `stream`.
tk_status launch_group(tk_tree* t, Lane* lane, const Plan* plan, Group& gr, const StitchArgs& base,
                       hipStream_t stream) {
  const int64_t nj = int64_t(gr.jobs.size());
  if (nj == 0) return TK_OK;
  const size_t lds_bytes = size_t(gr.lds_doubles) * 8;
  const int per_cu = t->tuning.persistent ? stitch_blocks_per_cu(gr.threads, lds_bytes) : 0;
  DevBuf* ws = &lane->ws[gr.bin];
  DevBuf* djobs = &lane->jobs[gr.bin];
  int64_t i0 = 0;
  while (i0 < nj) {
    const int64_t base_off = gr.jobs[size_t(i0)].ws_off;
    int64_t i1 = i0 + 1;
    while (i1 < nj && i1 - i0 < kMaxJobsPerLaunch &&
           gr.jobs[size_t(i1)].ws_off + gr.jobs[size_t(i1)].ws_bytes - base_off <= kWsChunkBytes)
      ++i1;
    if (i0 > 0) TK_HIP(t, hipStreamSynchronize(stream));  // the buffers are reused by this chunk
    const int64_t bytes = gr.jobs[size_t(i1 - 1)].ws_off + gr.jobs[size_t(i1 - 1)].ws_bytes - base_off;
    tk_status st = ensure(t, ws, bytes + 256, "workspace");
    if (st) return st;
    std::vector<Job> chunk(gr.jobs.begin() + i0, gr.jobs.begin() + i1);
    for (Job& jb : chunk) jb.ws_off -= base_off;
    st = ensure(t, djobs, int64_t(chunk.size() * sizeof(Job)), "jobs");
    if (st) return st;
    TK_HIP(t, hipMemcpyAsync(djobs->p, chunk.data(), chunk.size() * sizeof(Job), hipMemcpyHostToDevice, stream));
    std::vector<TrimChunk> trims;
    trim_chunks_of(t, *plan, gr, i0, i1, ws->p, trims);
    if (!trims.empty()) {  // the trim pass: row Grams of the long partial hits
      st = ensure(t, &lane->trims[gr.bin], int64_t(trims.size() * sizeof(TrimChunk)), "trim chunks");
      if (st) return st;
      TK_HIP(t, hipMemcpyAsync(lane->trims[gr.bin].p, trims.data(), trims.size() * sizeof(TrimChunk),
                               hipMemcpyHostToDevice, stream));
      TK_HIP(t, launch_trim(reinterpret_cast<const TrimChunk*>(lane->trims[gr.bin].p), int64_t(trims.size()), stream));
    }
    StitchArgs a = base;
    a.jobs = reinterpret_cast<const Job*>(djobs->p);
    a.ws = ws->p;
    a.n_jobs = int(i1 - i0);
    a.n_lds = gr.n_lds;
    a.lds_doubles = gr.lds_doubles;
    int grid = a.n_jobs;
    if (per_cu > 0) {
      const int64_t res = int64_t(per_cu) * t->n_cu;
      if (res < grid) grid = int(res);
      a.queue = reinterpret_cast<int*>(lane->queue.p) + gr.bin;
      TK_HIP(t, launch_reset_queue(a.queue, 1, stream));
    } else {
      a.queue = nullptr;
    }
    TK_HIP(t, launch_stitch(a, grid, lds_bytes, gr.threads, stream));
    i0 = i1;
  }
  return TK_OK;
}

}  // namespace

tk_status run_plan(tk_tree* t, Lane* lane, Plan& plan, int max_iter, double tol, bool fork) {
  if (plan.n_jobs == 0) return TK_OK;
  tk_status st = ensure(t, &lane->hits, int64_t(plan.hits.size() * sizeof(Hit)) + 64, "hits");
  if (st) return st;
  st = ensure(t, &lane->queue, kMaxGroups * 64, "queue");
  if (st) return st;
  if (!plan.hits.empty())
    TK_HIP(t, hipMemcpyAsync(lane->hits.p, plan.hits.data(), plan.hits.size() * sizeof(Hit), hipMemcpyHostToDevice,
                             lane->stream));
  StitchArgs base = stitch_args(t, max_iter, tol);
  base.basis_pct = plan.basis_pct;
  base.hits = reinterpret_cast<Hit*>(lane->hits.p);
  if (!fork || plan.groups.size() <= 1) {
    for (Group& gr : plan.groups) {
      st = launch_group(t, lane, &plan, gr, base, lane->stream);
      if (st) return st;
    }
    return TK_OK;
  }
  if (!lane->fork_ev) TK_HIP(t, hipEventCreateWithFlags(&lane->fork_ev, hipEventDisableTiming));
  TK_HIP(t, hipEventRecord(lane->fork_ev, lane->stream));
  bool used[kForkStreams] = {false, false, false, false};
  for (Group& gr : plan.groups) {
    const int sl = gr.slot;
    if (!lane->gstream[sl]) {
      TK_HIP(t, hipStreamCreateWithFlags(&lane->gstream[sl], hipStreamNonBlocking));
      TK_HIP(t, hipEventCreateWithFlags(&lane->gev[sl], hipEventDisableTiming));
    }
    if (!used[sl]) TK_HIP(t, hipStreamWaitEvent(lane->gstream[sl], lane->fork_ev, 0));
    used[sl] = true;
    st = launch_group(t, lane, &plan, gr, base, lane->gstream[sl]);
    if (st) return st;
  }
  // join only after every group is queued (a join between launches would
  // hold back the groups queued behind it)
  for (int sl = 0; sl < kForkStreams; ++sl) {
    if (!used[sl]) continue;
    TK_HIP(t, hipEventRecord(lane->gev[sl], lane->gstream[sl]));
    TK_HIP(t, hipStreamWaitEvent(lane->stream, lane->gev[sl], 0));
  }
  return TK_OK;
}

namespace {

int nu2_trailing_ones(int64_t b) {
  int n = 0;
  while (b & 1) {
    ++n;
    b >>= 1;
  }
  return n;
}

tk_status run_leaves(tk_tree* t, Lane* lane, int64_t first_block, int64_t nb, const float* X) {
  if (nb <= 0) return TK_OK;
  LeafLayout lo;
  leaf_layout(t->view, 1 << 30, &lo);
  int cap = 128;
  while (cap > 8 && int64_t(eig_doubles(cap)) * 8 > t->lds_limit - int64_t(leaf_static_lds())) cap -= 8;
  const int n_lds = lo.neig < cap ? lo.neig : cap;
  leaf_layout(t->view, n_lds, &lo);
  const size_t lds_bytes = size_t(eig_doubles(n_lds)) * 8;
  const int64_t per = lo.total;
  int64_t chunk = kWsChunkBytes / (per > 0 ? per : 1);
  if (chunk < 1) chunk = 1;
  if (chunk > kMaxJobsPerLaunch) chunk = kMaxJobsPerLaunch;
  const int64_t block_elems = t->ell * t->slice_elems;
  for (int64_t i0 = 0; i0 < nb; i0 += chunk) {
    const int64_t n = (nb - i0) < chunk ? (nb - i0) : chunk;
    if (i0 > 0) TK_HIP(t, hipStreamSynchronize(lane->stream));  // jobs/ws are reused by this chunk
    tk_status st = ensure(t, &lane->leaf_ws, n * per + 256, "workspace");
    if (st) return st;
    std::vector<LeafJob> jobs(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
      jobs[i].X = X + (i0 + i) * block_elems;
      jobs[i].block = first_block + i0 + i;
      jobs[i].stats = nullptr;
      jobs[i].ws_off = i * per;
    }
    st = ensure(t, &lane->leaf_jobs, n * int64_t(sizeof(LeafJob)), "jobs");
    if (st) return st;
    TK_HIP(t, hipMemcpyAsync(lane->leaf_jobs.p, jobs.data(), size_t(n) * sizeof(LeafJob), hipMemcpyHostToDevice,
                             lane->stream));
    LeafArgs a;
    a.st = t->dview;
    a.jobs = reinterpret_cast<const LeafJob*>(lane->leaf_jobs.p);
    a.ws = lane->leaf_ws.p;
    a.n_lds = n_lds;
    a.max_iter = t->cfg.max_iter;
    a.tol = t->cfg.tol;
    TK_HIP(t, launch_leaf(a, int(n), lds_bytes, lane->stream));
  }
  return TK_OK;
}

}  // namespace

tk_status commit_blocks(tk_tree* t, Lane* lane, int64_t nb, const float* Xdev, hipEvent_t* lev_ev, int n_ev) {
  const int64_t b0 = t->Tb, b1 = t->Tb + nb;
  tk_status st = run_leaves(t, lane, b0, nb, Xdev);
  if (st) return st;
  if (lev_ev && n_ev > 0) TK_HIP(t, hipEventRecord(lev_ev[0], lane->stream));
  const int K = root_level(b1);
  int64_t merges = 0;
  for (int k = 1; k <= K; ++k) {
    // nodes (k, j) with (j+1) 2^k in (b0, b1]
    const int64_t jlo = b0 >> k;
    const int64_t jhi = (b1 >> k) - 1;
    if (jhi < jlo) {
      if (lev_ev && k < n_ev) TK_HIP(t, hipEventRecord(lev_ev[k], lane->stream));
      continue;
    }
    std::vector<Job> jobs;
    std::vector<Hit> hits;
    for (int64_t j = jlo; j <= jhi; ++j) make_merge_job(t, k, j, jobs, hits);
    merges += int64_t(jobs.size());
    Plan plan;
    st = plan_stitch(t, jobs, hits, &plan);
    if (st) return st;
    // a commit's levels run one after another, each as long as its slowest
    // merge, so a merge's latency sets the commit time: at least two
    // wavefronts a merge (the thread count stays a function of the job and
    // the tuning, so appends and builds store the same bits)
    for (Group& gr : plan.groups) gr.threads = std::max(gr.threads, kMergeThreads);
    // one level's merges share a shape; groups run in order on the lane
    st = run_plan(t, lane, plan, t->cfg.max_iter, t->cfg.tol, false);
    if (st) return st;
    if (lev_ev && k < n_ev) TK_HIP(t, hipEventRecord(lev_ev[k], lane->stream));
  }
  t->Tb = b1;
  t->merges_total += merges;
  t->merges_last = nu2_trailing_ones(b1 - 1);
  return TK_OK;
}

}  // namespace tk

using namespace tk;

namespace {

bool range_ok(const tk_tree* t, int64_t ts, int64_t te) {
  return ts >= 0 && ts < te && te <= t->Tb * t->ell;
}

tk_status busy(tk_tree* t) { return fail(t, TK_EBUSY, "the tree is serving; stop the server first"); }

}  // namespace

extern "C" {

const char* tk_version(void) { return "0.1.0"; }

const char* tk_last_error(const tk_tree* t) {
  if (!t) return g_create_error.c_str();
  // a per-thread copy: another thread may replace the tree's text meanwhile
  thread_local std::string copy;
  std::lock_guard<std::mutex> lk(t->err_mu);
  copy = t->err;
  return copy.c_str();
}

tk_status tk_create(const tk_config* cfg, void* hip_stream, tk_tree** out) {
  if (!cfg || !out) return fail(nullptr, TK_EINVAL, "null argument");
  *out = nullptr;
  const int p = cfg->p;
  if (p < 2 || p > tk::MAXP) return fail(nullptr, TK_EINVAL, "p must be in [2, 7]");
  int64_t slice = 1;
  for (int n = 1; n < p; ++n) {
    if (cfg->dims[n] < 1 || cfg->dims[n] > (1 << 20)) return fail(nullptr, TK_EINVAL, "bad dims");
    slice *= cfg->dims[n];
    if (slice > (int64_t(1) << 30)) return fail(nullptr, TK_EINVAL, "slice too large");
  }
  for (int n = 0; n < p; ++n)
    if (cfg->ranks[n] < 1 || cfg->ranks[n] > kMaxRank) return fail(nullptr, TK_EINVAL, "ranks must be in [1, 32]");
  if (cfg->leaf_len < 1 || cfg->leaf_len > (1 << 16)) return fail(nullptr, TK_EINVAL, "bad leaf_len");
  if (int64_t(cfg->leaf_len) * slice > (int64_t(1) << 30)) return fail(nullptr, TK_EINVAL, "leaf block too large");
  if (cfg->theta_num < 1 || cfg->theta_den < cfg->theta_num || cfg->theta_den > (1 << 20))
    return fail(nullptr, TK_EINVAL, "theta must be num/den in (0, 1]");
  if (cfg->max_iter < 1 || cfg->max_iter > 100000) return fail(nullptr, TK_EINVAL, "bad max_iter");
  if (!(cfg->tol >= 0.0) || !std::isfinite(cfg->tol)) return fail(nullptr, TK_EINVAL, "bad tol");
  if (cfg->prec != TK_F32 && cfg->prec != TK_BF16) return fail(nullptr, TK_EINVAL, "prec must be TK_F32 or TK_BF16");
  if (cfg->capacity_T < cfg->leaf_len || cfg->capacity_T > (int64_t(1) << 40))
    return fail(nullptr, TK_EINVAL, "bad capacity_T");

  tk_tree* t = new tk_tree();
  t->cfg = *cfg;
  t->stream = static_cast<hipStream_t>(hip_stream);
  t->main.stream = t->stream;
  t->p = p;
  t->ell = cfg->leaf_len;
  t->slice_elems = slice;
  t->cap_blocks = cfg->capacity_T / cfg->leaf_len;
  t->nlev = tk::root_level(t->cap_blocks) + 1;
  t->q_max_iter = cfg->max_iter;
  t->q_tol = cfg->tol;
  t->q_prec = cfg->prec;
  StoreView& v = t->view;
  v.p = p;
  v.nlev = t->nlev;
  v.ell = t->ell;
  for (int n = 0; n < tk::MAXP; ++n) v.D[n] = n < p && n > 0 ? cfg->dims[n] : 0;
  // sizes
  int64_t off = 0;
  std::vector<int64_t> o_core(t->nlev), o_plane(t->nlev), o_fac(size_t(t->nlev) * tk::MAXP, 0);
  for (int k = 0; k < t->nlev; ++k) {
    tk::effective_ranks(p, t->ell << k, v.D, cfg->ranks, v.rk[k]);
    int64_t ce = 1;
    for (int n = 0; n < p; ++n) ce *= v.rk[k][n];
    v.core_elems[k] = ce;
    const int64_t nk = (t->cap_blocks + (int64_t(1) << k) - 1) >> k;
    o_core[k] = off;
    off = tk::align256(off + nk * ce * 4);
    for (int n = 1; n < p; ++n) {
      o_fac[size_t(k) * tk::MAXP + n] = off;
      off = tk::align256(off + nk * v.D[n] * v.rk[k][n] * 4);
    }
    o_plane[k] = off;
    off = tk::align256(off + t->cap_blocks * t->ell * v.rk[k][0] * 4);
  }
  t->store_bytes = off;
  const int64_t block_bytes = t->ell * slice * 4;
  if (cfg->mem_budget_bytes > 0 && t->store_bytes + block_bytes > cfg->mem_budget_bytes) {
    delete t;
    return fail(nullptr, TK_ENOMEM, "node store exceeds mem_budget_bytes");
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    delete t;
    return fail_dev(nullptr, e, "hipGetDevice");
  }
  t->device = dev;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      t->n_cu = ncu;
  }
  void* ptr = nullptr;
  e = hipMalloc(&ptr, size_t(t->store_bytes));
  if (e != hipSuccess) {
    delete t;
    return fail_dev(nullptr, e, "hipMalloc(node store)");
  }
  t->store = static_cast<char*>(ptr);
  for (int k = 0; k < t->nlev; ++k) {
    v.core[k] = reinterpret_cast<float*>(t->store + o_core[k]);
    v.plane[k] = reinterpret_cast<float*>(t->store + o_plane[k]);
    for (int n = 0; n < tk::MAXP; ++n)
      v.fac[k][n] = (n >= 1 && n < p) ? reinterpret_cast<float*>(t->store + o_fac[size_t(k) * tk::MAXP + n])
                                      : nullptr;
  }
  const char* step = "hipMalloc(store view)";
  e = hipMalloc(&ptr, sizeof(StoreView));
  if (e == hipSuccess) {
    t->dview = static_cast<StoreView*>(ptr);
    step = "hipMalloc(block buffer)";
    e = hipMalloc(&ptr, size_t(block_bytes));
  }
  if (e == hipSuccess) {
    t->block_buf = static_cast<float*>(ptr);
    step = "hipMemsetAsync(node store)";
    e = hipMemsetAsync(t->store, 0, size_t(t->store_bytes), t->stream);
  }
  if (e == hipSuccess) {
    step = "hipMemcpyAsync(store view)";
    e = hipMemcpyAsync(t->dview, &t->view, sizeof(StoreView), hipMemcpyHostToDevice, t->stream);
  }
  if (e == hipSuccess) {
    // dynamic LDS per workgroup: the device's opt-in limit, at most 160 KiB,
    // stepping down if the runtime refuses a request
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess ||
        optin <= 0) {
      optin = 0;
      (void)hipDeviceGetAttribute(&optin, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    }
    int64_t lim = optin > 0 && optin < int(kLdsBytes) ? optin : int64_t(kLdsBytes);
    step = "hipFuncSetAttribute(MaxDynamicSharedMemorySize)";
    e = hipErrorInvalidValue;
    while (lim >= 32768) {
      e = tk::set_lds_limits(size_t(lim) - tk::stitch_static_lds(), size_t(lim) - tk::leaf_static_lds());
      if (e == hipSuccess) break;
      (void)hipGetLastError();
      lim -= 16384;
    }
    t->lds_limit = lim;
  }
  if (e == hipSuccess) {
    step = "hipGetSymbolAddress(no-allocation scratch)";
    (void)tk::noalloc_scratch(dev, &e);
  }
  if (e == hipSuccess) {
    step = "hipStreamSynchronize(create)";
    e = hipStreamSynchronize(t->stream);
  }
  if (e != hipSuccess) {
    tk_status st = fail_dev(nullptr, e, step);
    tk_destroy(t);
    return st;
  }
  *out = t;
  return TK_OK;
}

void tk_destroy(tk_tree* t) {
  if (!t) return;
  tk_serve_stop(t);
  (void)hipStreamSynchronize(t->stream);
  lane_destroy(&t->main);
  if (t->store) (void)hipFree(t->store);
  if (t->dview) (void)hipFree(t->dview);
  if (t->block_buf) (void)hipFree(t->block_buf);
  tk::release(&t->prov_out);
  if (t->ev0) (void)hipEventDestroy(t->ev0);
  if (t->ev1) (void)hipEventDestroy(t->ev1);
  delete t;
}

tk_status tk_append(tk_tree* t, const float* slice, int on_device) {
  if (!t || !slice) return fail(t, TK_EINVAL, "null argument");
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  if (t->T >= t->cap_blocks * t->ell) return fail(t, TK_ENOMEM, "capacity_T reached");
  const int64_t row = t->T % t->ell;
  TK_HIP(t, hipMemcpyAsync(t->block_buf + row * t->slice_elems, slice, size_t(t->slice_elems) * 4,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, t->stream));
  if (row == t->tail_rows) t->tail_rows = row + 1;
  t->T += 1;
  if (t->T % t->ell == 0) {
    tk_status st = commit_blocks(t, &t->main, 1, t->block_buf);
    if (st) return st;
    TK_HIP(t, hipStreamSynchronize(t->stream));
    t->tail_rows = 0;
  }
  return TK_OK;
}

tk_status tk_build(tk_tree* t, const float* X, int64_t T, int on_device) {
  if (!t || (!X && T > 0) || T < 0) return fail(t, TK_EINVAL, "bad argument");
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  if (t->T + T > t->cap_blocks * t->ell) return fail(t, TK_ENOMEM, "capacity_T exceeded");
  int64_t done = 0;
  if (t->T % t->ell == 0) {
    const int64_t nb = T / t->ell;
    const int64_t block_elems = t->ell * t->slice_elems;
    if (nb > 0) {
      const float* Xd = X;
      if (!on_device) {
        tk_status st = ensure(t, &t->main.xbuf, nb * block_elems * 4, "staging");
        if (st) return st;
        TK_HIP(t, hipMemcpyAsync(t->main.xbuf.p, X, size_t(nb * block_elems) * 4, hipMemcpyHostToDevice, t->stream));
        Xd = reinterpret_cast<const float*>(t->main.xbuf.p);
      }
      tk_status st = commit_blocks(t, &t->main, nb, Xd);
      if (st) return st;
      t->T += nb * t->ell;
      done = nb * t->ell;
    }
  }
  for (int64_t s = done; s < T; ++s) {
    tk_status st = tk_append(t, X + s * t->slice_elems, on_device);
    if (st) return st;
  }
  TK_HIP(t, hipStreamSynchronize(t->stream));
  return TK_OK;
}

tk_status tk_hitset(const tk_tree* t, int64_t ts, int64_t te, tk_hit* out, int32_t cap, int32_t* n) {
  if (!t || !n || (cap > 0 && !out)) return TK_EINVAL;
  if (t->server) return TK_EBUSY;
  if (!range_ok(t, ts, te)) return TK_ERANGE;
  Hit buf[tk::MAXHITS];
  const int m = tk::query_hits(t, ts, te, t->Tb, buf, tk::MAXHITS);
  *n = m;
  for (int i = 0; i < m && i < cap && i < tk::MAXHITS; ++i) {
    const int64_t sig = (buf[i].index << buf[i].level) * t->ell;
    out[i].level = buf[i].level;
    out[i].index = buf[i].index;
    out[i].partial = buf[i].partial;
    out[i].node_id = tk::node_id(buf[i].level, buf[i].index);
    out[i].sigma = sig;
    out[i].tau = sig + (t->ell << buf[i].level);
    out[i].lo = sig + buf[i].a;
    out[i].hi = sig + buf[i].a + buf[i].l;
  }
  return TK_OK;
}

tk_status tk_query_shape(const tk_tree* t, int64_t ts, int64_t te, tk_shape* out) {
  if (!t || !out) return TK_EINVAL;
  if (t->server) return TK_EBUSY;
  Hit buf[tk::MAXHITS];
  bool tail = false;
  const int nh = tk::plan_query_hits(t, ts, te, t->Tb, true, buf, tk::MAXHITS, &tail);
  if (nh < 0) return TK_ERANGE;
  if (nh > tk::MAXHITS) return TK_EINVAL;
  std::memset(out, 0, sizeof(*out));
  tk::query_ranks(t, te - ts, out->ranks_eff);
  out->L = te - ts;
  out->core_elems = 1;
  for (int n = 0; n < t->p; ++n) out->core_elems *= out->ranks_eff[n];
  out->factor_elems[0] = out->L * out->ranks_eff[0];
  for (int n = 1; n < t->p; ++n) out->factor_elems[n] = t->view.D[n] * out->ranks_eff[n];
  out->n_hits = nh;
  tk::StitchLayout lo;
  tk::stitch_layout(t->view, buf, out->n_hits, out->ranks_eff, 0, &lo);
  out->ws_bytes = lo.total;
  return TK_OK;
}

tk_status tk_query_batch(tk_tree* t, int32_t n, const int64_t* ts, const int64_t* te, tk_result* res) {
  if (!t || n < 0 || (n > 0 && (!ts || !te || !res))) return fail(t, TK_EINVAL, "bad argument");
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  std::vector<Job> jobs;
  std::vector<Hit> hits;
  jobs.reserve(size_t(n));
  bool any_tail = false;
  for (int32_t i = 0; i < n; ++i) {
    tk_status st = make_query_job(t, ts[i], te[i], t->Tb, &res[i], true, jobs, hits, true);
    if (st) return st;
    any_tail = any_tail || te[i] > t->Tb * t->ell;
  }
  if (n == 0) return TK_OK;
  if (any_tail) {
    tk_status st = provisional_leaf(t);
    if (st) return st;
  }
  tk_status st = ensure(t, &t->main.stats, int64_t(n) * STAT_COUNT * 8, "stats");
  if (st) return st;
  double* dstats = reinterpret_cast<double*>(t->main.stats.p);
  for (int32_t i = 0; i < n; ++i) jobs[i].stats = dstats + STAT_COUNT * int64_t(i);
  Plan plan;
  st = plan_stitch(t, jobs, hits, &plan);
  if (st) return st;
  if (!t->ev0) {
    TK_HIP(t, hipEventCreate(&t->ev0));
    TK_HIP(t, hipEventCreate(&t->ev1));
  }
  t->ev_valid = false;
  TK_HIP(t, hipEventRecord(t->ev0, t->stream));
  st = run_plan(t, &t->main, plan, t->q_max_iter, t->q_tol, true);
  if (st) return st;
  TK_HIP(t, hipEventRecord(t->ev1, t->stream));
  t->ev_valid = true;
  std::vector<double>& hs = t->last_stats;
  hs.assign(size_t(n) * STAT_COUNT, 0.0);
  TK_HIP(t, hipMemcpyAsync(hs.data(), dstats, hs.size() * 8, hipMemcpyDeviceToHost, t->stream));
  TK_HIP(t, hipStreamSynchronize(t->stream));
  for (int32_t i = 0; i < n; ++i) {
    const double* s = hs.data() + STAT_COUNT * size_t(i);
    if (s[STAT_STATUS] != 0.0)
      return fail(t, TK_EDEVICE, job_status_msg(s[STAT_STATUS]));
    for (int m = 0; m < TK_MAX_MODES; ++m) res[i].ranks_eff[m] = m < t->p ? jobs[i].rq[m] : 0;
    res[i].fit = s[STAT_FIT];
    res[i].err_model = s[STAT_ERR];
    res[i].norm_ytilde = s[STAT_NORM];
    res[i].sweeps = int32_t(s[STAT_SWEEPS]);
    res[i].converged = int32_t(s[STAT_CONV]);
    res[i].n_hits = jobs[i].s;
  }
  return TK_OK;
}

tk_status tk_query(tk_tree* t, int64_t ts, int64_t te, tk_result* res) {
  return tk_query_batch(t, 1, &ts, &te, res);
}

tk_status tk_query_noalloc(tk_tree* t, int64_t ts, int64_t te, tk_result* res) {
  using namespace tk;
  if (!t || !res) return fail(t, TK_EINVAL, "bad argument");
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  if (!(ts >= 0 && ts < te && te <= t->Tb * t->ell))
    return fail(t, TK_ERANGE, "query range outside [0, T_c) or empty (no ranges into the incomplete block here)");
  std::vector<Job> jobs;
  std::vector<Hit> hits;
  tk_status st = make_query_job(t, ts, te, t->Tb, res, true, jobs, hits, false);
  if (st) return st;
  Plan plan;
  st = plan_stitch(t, jobs, hits, &plan);
  if (st) return st;
  if (plan.groups.size() != 1 || plan.groups[0].jobs.size() != 1) return fail(t, TK_EINVAL, "one query, one job");
  const Group& gr = plan.groups[0];
  // scratch layout: hits | queue counters | stats | job descriptor | workspace
  const int64_t o_hits = 0;
  const int64_t o_queue = align256(o_hits + int64_t(plan.hits.size() * sizeof(Hit)) + 64);
  const int64_t o_stats = align256(o_queue + kMaxGroups * 64);
  const int64_t o_jobs = align256(o_stats + STAT_COUNT * 8);
  const int64_t o_ws = align256(o_jobs + int64_t(sizeof(Job)));
  const int64_t ws_cap = kNoAllocScratchBytes - o_ws;
  if (gr.ws_total + 256 > ws_cap)
    return fail(t, TK_ENOMEM, "the query's workspace (" + std::to_string(gr.ws_total) +
                                  " bytes) exceeds the no-allocation scratch (" + std::to_string(ws_cap) + " bytes)");
  hipError_t e = hipSuccess;
  char* base = noalloc_scratch(t->device, &e);
  if (!base) return fail_dev(t, e, "no-allocation scratch address");
  // a lane whose buffers all lie in the scratch (fixed: never reallocated)
  Lane lane;
  lane.stream = t->stream;
  auto fix = [&](DevBuf* b, int64_t off, int64_t cap) {
    b->p = base + off;
    b->cap = cap;
    b->fixed = true;
  };
  fix(&lane.hits, o_hits, o_queue - o_hits);
  fix(&lane.queue, o_queue, o_stats - o_queue);
  fix(&lane.stats, o_stats, o_jobs - o_stats);
  for (int g = 0; g < kMaxGroups; ++g) {
    fix(&lane.jobs[g], o_jobs, o_ws - o_jobs);
    fix(&lane.ws[g], o_ws, ws_cap);
  }
  double* dstats = reinterpret_cast<double*>(lane.stats.p);
  plan.groups[0].jobs[0].stats = dstats;
  st = run_plan(t, &lane, plan, t->q_max_iter, t->q_tol, false);
  if (st) return st;
  double hs[STAT_COUNT];
  TK_HIP(t, hipMemcpyAsync(hs, dstats, sizeof(hs), hipMemcpyDeviceToHost, t->stream));
  TK_HIP(t, hipStreamSynchronize(t->stream));
  if (hs[STAT_STATUS] != 0.0) return fail(t, TK_EDEVICE, job_status_msg(hs[STAT_STATUS]));
  for (int m = 0; m < TK_MAX_MODES; ++m) res->ranks_eff[m] = m < t->p ? jobs[0].rq[m] : 0;
  res->fit = hs[STAT_FIT];
  res->err_model = hs[STAT_ERR];
  res->norm_ytilde = hs[STAT_NORM];
  res->sweeps = int32_t(hs[STAT_SWEEPS]);
  res->converged = int32_t(hs[STAT_CONV]);
  res->n_hits = jobs[0].s;
  return TK_OK;
}

tk_status tk_raw_tucker(tk_tree* t, int32_t n, const float* const* X, const int64_t* L, tk_result* res) {
  using namespace tk;
  if (!t || n < 0 || (n > 0 && (!X || !L || !res))) return TK_EINVAL;
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  if (n == 0) return TK_OK;
  const int p = t->p;
  int cap = 128;
  while (cap > 8 && int64_t(eig_doubles(cap)) * 8 > t->lds_limit - int64_t(leaf_static_lds())) cap -= 8;
  std::vector<RawJob> jobs(static_cast<size_t>(n));
  int neig = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!X[i] || L[i] < 1 || L[i] > (int64_t(1) << 30)) return fail(t, TK_EINVAL, "raw range: null data or bad length");
    if (!res[i].core) return fail(t, TK_EINVAL, "null core buffer");
    RawJob& jb = jobs[size_t(i)];
    jb = RawJob{};
    jb.X = X[i];
    jb.L = L[i];
    query_ranks(t, L[i], jb.rq);
    jb.out_core = res[i].core;
    for (int m = 0; m < p; ++m) {
      if (!res[i].factor[m]) return fail(t, TK_EINVAL, "null factor buffer");
      jb.out_fac[m] = res[i].factor[m];
    }
    int32_t Dm[MAXP];
    Dm[0] = int32_t(L[i]);
    for (int m = 1; m < p; ++m) Dm[m] = int32_t(t->view.D[m]);
    LeafLayout lo;
    raw_layout(p, Dm, jb.rq, 1 << 30, &lo);
    if (lo.neig > EIG_MAXK_HOST) return fail(t, TK_EINVAL, "raw range needs an eigenproblem above 1024");
    if (lo.neig > neig) neig = lo.neig;
  }
  const int n_lds = neig < cap ? neig : cap;
  const size_t lds_bytes = size_t(eig_doubles(n_lds)) * 8;
  std::vector<int64_t> bytes(static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i) {
    int32_t Dm[MAXP];
    Dm[0] = int32_t(L[i]);
    for (int m = 1; m < p; ++m) Dm[m] = int32_t(t->view.D[m]);
    LeafLayout lo;
    raw_layout(p, Dm, jobs[size_t(i)].rq, n_lds, &lo);
    bytes[size_t(i)] = lo.total;
  }
  Lane* lane = &t->main;
  tk_status st = ensure(t, &lane->stats, int64_t(n) * STAT_COUNT * 8, "stats");
  if (st) return st;
  TK_HIP(t, hipMemsetAsync(lane->stats.p, 0, size_t(n) * STAT_COUNT * 8, lane->stream));
  double* dstats = reinterpret_cast<double*>(lane->stats.p);
  RawArgs a{};
  a.p = p;
  for (int m = 1; m < p; ++m) a.D[m] = int32_t(t->view.D[m]);
  a.n_lds = n_lds;
  a.max_iter = t->q_max_iter;
  a.tol = t->q_tol;
  int32_t i0 = 0;
  while (i0 < n) {
    int64_t ws = 0;
    int32_t i1 = i0;
    while (i1 < n && i1 - i0 < kMaxJobsPerLaunch && (i1 == i0 || ws + bytes[size_t(i1)] <= kWsChunkBytes)) {
      jobs[size_t(i1)].ws_off = ws;
      jobs[size_t(i1)].stats = dstats + STAT_COUNT * int64_t(i1);
      ws += bytes[size_t(i1)];
      ++i1;
    }
    if (i0 > 0) TK_HIP(t, hipStreamSynchronize(lane->stream));  // buffers are reused by this chunk
    st = ensure(t, &lane->leaf_ws, ws + 256, "workspace");
    if (st) return st;
    st = ensure(t, &lane->leaf_jobs, int64_t(i1 - i0) * int64_t(sizeof(RawJob)), "jobs");
    if (st) return st;
    TK_HIP(t, hipMemcpyAsync(lane->leaf_jobs.p, jobs.data() + i0, size_t(i1 - i0) * sizeof(RawJob),
                             hipMemcpyHostToDevice, lane->stream));
    a.jobs = reinterpret_cast<const RawJob*>(lane->leaf_jobs.p);
    a.ws = lane->leaf_ws.p;
    TK_HIP(t, launch_raw(a, i1 - i0, lds_bytes, lane->stream));
    i0 = i1;
  }
  std::vector<double> hs(size_t(n) * STAT_COUNT, 0.0);
  TK_HIP(t, hipMemcpyAsync(hs.data(), dstats, hs.size() * 8, hipMemcpyDeviceToHost, lane->stream));
  TK_HIP(t, hipStreamSynchronize(lane->stream));
  for (int32_t i = 0; i < n; ++i) {
    const double* s = hs.data() + STAT_COUNT * size_t(i);
    for (int m = 0; m < TK_MAX_MODES; ++m) res[i].ranks_eff[m] = m < p ? jobs[size_t(i)].rq[m] : 0;
    res[i].fit = s[STAT_FIT];
    res[i].err_model = s[STAT_ERR];
    res[i].norm_ytilde = s[STAT_NORM];
    res[i].sweeps = int32_t(s[STAT_SWEEPS]);
    res[i].converged = int32_t(s[STAT_CONV]);
    res[i].n_hits = 0;
  }
  return TK_OK;
}

tk_status tk_last_query_kernel_ms(const tk_tree* t, double* ms) {
  if (!t || !ms) return TK_EINVAL;
  if (!t->ev_valid) return TK_EINVAL;
  float f = 0.f;
  if (hipEventSynchronize(t->ev1) != hipSuccess) return TK_EDEVICE;
  if (hipEventElapsedTime(&f, t->ev0, t->ev1) != hipSuccess) return TK_EDEVICE;
  *ms = double(f);
  return TK_OK;
}

tk_status tk_last_query_profile(const tk_tree* t, int32_t i, double* phase_us) {
  if (!t || !phase_us || i < 0) return TK_EINVAL;
  const int64_t n = int64_t(t->last_stats.size()) / tk::STAT_COUNT;
  if (i >= n) return TK_EINVAL;
  for (int k = 0; k < tk::PROFILE_COUNT; ++k)
    phase_us[k] = t->last_stats[size_t(i) * tk::STAT_COUNT + tk::STAT_PHASE + k] *
                  (k == tk::STAT_NPHASE + 4 || k == tk::STAT_NPHASE + 5 ? 0.01 : 1.0);
  return TK_OK;
}

tk_status tk_set_query_iters(tk_tree* t, int32_t max_iter, double tol) {
  if (!t || max_iter < 1 || !(tol >= 0.0)) return TK_EINVAL;
  if (t->server) return busy(t);
  t->q_max_iter = max_iter;
  t->q_tol = tol;
  return TK_OK;
}

tk_status tk_set_query_prec(tk_tree* t, int32_t prec) {
  if (!t || (prec != TK_F32 && prec != TK_BF16)) return TK_EINVAL;
  if (t->server) return busy(t);
  t->q_prec = prec;
  return TK_OK;
}

tk_status tk_set_query_recall(tk_tree* t, int32_t level) {
  if (!t || level < -1 || level >= t->nlev) return TK_EINVAL;
  if (t->server) return busy(t);
  t->q_level = level;
  return TK_OK;
}

tk_status tk_set_query_ranks(tk_tree* t, const int32_t* ranks) {
  if (!t) return TK_EINVAL;
  if (t->server) return busy(t);
  if (ranks)
    for (int n = 0; n < t->p; ++n)
      if (ranks[n] < 1 || ranks[n] > t->cfg.ranks[n]) return fail(t, TK_EINVAL, "query ranks must be in [1, cfg.ranks]");
  for (int n = 0; n < TK_MAX_MODES; ++n) t->q_ranks[n] = ranks && n < t->p ? ranks[n] : 0;
  return TK_OK;
}

tk_status tk_get_tuning(const tk_tree* t, tk_tuning* out) {
  if (!t || !out) return TK_EINVAL;
  out->wide_threshold = t->tuning.wide_threshold;
  out->wide_threads = t->tuning.wide_threads;
  out->persistent = t->tuning.persistent;
  out->graph = t->tuning.graph;
  out->coarse = t->tuning.coarse;
  out->lds_n = t->tuning.lds_n;
  out->basis_pct = t->tuning.basis_pct;
  out->rest_threads = t->tuning.rest_threads;
  out->wide_core = t->tuning.wide_core;
  return TK_OK;
}

tk_status tk_set_tuning(tk_tree* t, const tk_tuning* in) {
  if (!t || !in) return TK_EINVAL;
  if (t->server) return busy(t);
  if (in->wide_threshold < 16 || in->wide_threshold > EIG_MAXK_HOST)
    return fail(t, TK_EINVAL, "wide_threshold must be in [16, 1024]");
  if (in->wide_threads != 128 && in->wide_threads != 256) return fail(t, TK_EINVAL, "wide_threads must be 128 or 256");
  if (in->persistent != 0 && in->persistent != 1) return fail(t, TK_EINVAL, "persistent must be 0 or 1");
  if (in->graph != 0 && in->graph != 1) return fail(t, TK_EINVAL, "graph must be 0 or 1");
  if (in->coarse != 0 && in->coarse != 1) return fail(t, TK_EINVAL, "coarse must be 0 or 1");
  if (in->lds_n != 0 && (in->lds_n < 16 || in->lds_n < in->wide_threshold))
    return fail(t, TK_EINVAL, "lds_n must be 0 or in [max(16, wide_threshold), ...]");
  if (in->basis_pct < 1 || in->basis_pct > 100) return fail(t, TK_EINVAL, "basis_pct must be in [1, 100]");
  if (in->rest_threads != 0 && in->rest_threads != 128 && in->rest_threads != 256)
    return fail(t, TK_EINVAL, "rest_threads must be 0, 128 or 256");
  if (in->wide_core < 0) return fail(t, TK_EINVAL, "wide_core must be >= 0");
  t->tuning.wide_threshold = in->wide_threshold;
  t->tuning.wide_threads = in->wide_threads;
  t->tuning.persistent = in->persistent;
  t->tuning.graph = in->graph;
  t->tuning.coarse = in->coarse;
  t->tuning.lds_n = in->lds_n;
  t->tuning.basis_pct = in->basis_pct;
  t->tuning.rest_threads = in->rest_threads;
  t->tuning.wide_core = in->wide_core;
  return TK_OK;
}

tk_status tk_stats_get(const tk_tree* t, tk_stats* out) {
  if (!t || !out) return TK_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->T = t->T;
  out->T_committed = t->Tb * t->ell;
  out->blocks = t->Tb;
  if (t->Tb > 0) {
    const int K = tk::root_level(t->Tb);
    for (int k = 0; k <= K; ++k) out->nodes += (t->Tb + (int64_t(1) << k) - 1) >> k;
    out->height = K + 1;
  }
  out->merges_total = t->merges_total;
  out->merges_last = t->merges_last;
  out->store_bytes = t->store_bytes;
  return TK_OK;
}

tk_status tk_node_ranks(const tk_tree* t, int32_t level, int32_t* ranks_eff) {
  if (!t || !ranks_eff || level < 0 || level >= t->nlev) return TK_EINVAL;
  for (int n = 0; n < TK_MAX_MODES; ++n) ranks_eff[n] = n < t->p ? t->view.rk[level][n] : 0;
  return TK_OK;
}

tk_status tk_read_node(tk_tree* t, int32_t level, int64_t index, float* core, float* const* factor) {
  if (!t || !core || !factor || level < 0 || level >= t->nlev || index < 0) return TK_EINVAL;
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  if (!tk::node_complete(level, index, t->Tb)) return fail(t, TK_ERANGE, "node not complete");
  for (int n = 0; n < t->p; ++n)
    if (!factor[n]) return TK_EINVAL;
  const StoreView& v = t->view;
  TK_HIP(t, hipStreamSynchronize(t->stream));
  TK_HIP(t, hipMemcpy(core, v.core[level] + index * v.core_elems[level], size_t(v.core_elems[level]) * 4,
                      hipMemcpyDeviceToHost));
  for (int n = 1; n < t->p; ++n)
    TK_HIP(t, hipMemcpy(factor[n], v.fac[level][n] + index * tk::fac_elems(v, level, n),
                        size_t(tk::fac_elems(v, level, n)) * 4, hipMemcpyDeviceToHost));
  const int64_t rows = t->ell << level;
  TK_HIP(t, hipMemcpy(factor[0], v.plane[level] + (index << level) * t->ell * v.rk[level][0],
                      size_t(rows * v.rk[level][0]) * 4, hipMemcpyDeviceToHost));
  return TK_OK;
}

tk_status tk_restore_begin(tk_tree* t, int64_t T) {
  if (!t || T < 0 || T > t->cap_blocks * t->ell) return TK_EINVAL;
  // the slices of an incomplete block are not part of any node: a horizon
  // inside a block could not be continued by later appends
  if (T % t->ell != 0) return fail(t, TK_EINVAL, "restore horizon must end at a leaf block boundary");
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  t->T = T;
  t->Tb = T / t->ell;
  t->tail_rows = 0;
  t->prov_T = -1;
  t->merges_total = 0;
  t->merges_last = 0;
  return TK_OK;
}

tk_status tk_load_node(tk_tree* t, int32_t level, int64_t index, const float* core,
                       const float* const* factor) {
  if (!t || !core || !factor || level < 0 || level >= t->nlev || index < 0) return TK_EINVAL;
  if (t->server) return busy(t);
  if (t->poisoned) return TK_EDEVICE;
  if (!tk::node_complete(level, index, t->Tb)) return fail(t, TK_ERANGE, "node not complete");
  for (int n = 0; n < t->p; ++n)
    if (!factor[n]) return TK_EINVAL;
  const StoreView& v = t->view;
  TK_HIP(t, hipMemcpyAsync(v.core[level] + index * v.core_elems[level], core, size_t(v.core_elems[level]) * 4,
                           hipMemcpyHostToDevice, t->stream));
  for (int n = 1; n < t->p; ++n)
    TK_HIP(t, hipMemcpyAsync(v.fac[level][n] + index * tk::fac_elems(v, level, n), factor[n],
                             size_t(tk::fac_elems(v, level, n)) * 4, hipMemcpyHostToDevice, t->stream));
  const int64_t rows = t->ell << level;
  TK_HIP(t, hipMemcpyAsync(v.plane[level] + (index << level) * t->ell * v.rk[level][0], factor[0],
                           size_t(rows * v.rk[level][0]) * 4, hipMemcpyHostToDevice, t->stream));
  TK_HIP(t, hipStreamSynchronize(t->stream));
  return TK_OK;
}

tk_status tk_hitset_plan(const tk_config* cfg, int64_t T, int64_t ts, int64_t te, tk_hit* out, int32_t cap,
                         int32_t* n) {
  if (!cfg || !n || (cap > 0 && !out) || cfg->leaf_len < 1 || cfg->theta_num < 1 ||
      cfg->theta_den < cfg->theta_num || cfg->theta_den > (1 << 20) || T < 0)
    return TK_EINVAL;
  const int64_t ell = cfg->leaf_len;
  const int64_t Tb = T / ell;
  if (!(ts >= 0 && ts < te && te <= Tb * ell)) return TK_ERANGE;
  Hit buf[tk::MAXHITS];
  const int m = tk::recall(ts, te, Tb, ell, cfg->theta_num, cfg->theta_den, buf, tk::MAXHITS);
  *n = m;
  for (int i = 0; i < m && i < cap && i < tk::MAXHITS; ++i) {
    const int64_t sig = (buf[i].index << buf[i].level) * ell;
    out[i].level = buf[i].level;
    out[i].index = buf[i].index;
    out[i].partial = buf[i].partial;
    out[i].node_id = tk::node_id(buf[i].level, buf[i].index);
    out[i].sigma = sig;
    out[i].tau = sig + (ell << buf[i].level);
    out[i].lo = sig + buf[i].a;
    out[i].hi = sig + buf[i].a + buf[i].l;
  }
  return TK_OK;
}

tk_status tk_effective_ranks(const tk_config* cfg, int64_t length, int32_t* ranks_eff) {
  if (!cfg || !ranks_eff || cfg->p < 2 || cfg->p > tk::MAXP || length < 1) return TK_EINVAL;
  int64_t D[tk::MAXP] = {0};
  for (int n = 1; n < cfg->p; ++n) D[n] = cfg->dims[n];
  int32_t r[tk::MAXP];
  tk::effective_ranks(cfg->p, length, D, cfg->ranks, r);
  for (int n = 0; n < TK_MAX_MODES; ++n) ranks_eff[n] = n < cfg->p ? r[n] : 0;
  return TK_OK;
}

}  // extern "C"
