// C ABI of the TUCKET engine: tree object, node store, append/build
// scheduling and query launches.  Integer work (which nodes, where they live)
// happens here on the host; every floating-point step runs in the kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tk_internal.hpp"
#include "tucket.h"

using tk::Hit;
using tk::Job;
using tk::LeafJob;
using tk::StoreView;

namespace {

thread_local std::string g_create_error;

constexpr int kMaxRank = 32;
constexpr int64_t kMaxJobsPerLaunch = 1 << 16;
constexpr int64_t kWsChunkBytes = int64_t(4) << 30;  // workspace per launch chunk
constexpr size_t kLdsBytes = 160 * 1024;              // LDS per CU on gfx950

}  // namespace

struct tk_tree {
  tk_config cfg{};
  hipStream_t stream = nullptr;
  int p = 0;
  int64_t ell = 1;
  int64_t cap_blocks = 0;
  int nlev = 0;
  StoreView view{};
  StoreView* dview = nullptr;
  char* store = nullptr;
  int64_t store_bytes = 0;
  float* block_buf = nullptr;
  int64_t slice_elems = 0;
  int64_t T = 0;
  int64_t Tb = 0;
  int64_t merges_total = 0;
  int64_t merges_last = 0;
  char* ws = nullptr;
  int64_t ws_cap = 0;
  char* djobs = nullptr;
  int64_t djobs_cap = 0;
  // per-bin launch resources: bins of a query batch run concurrently on
  // their own streams, joined back to the tree's stream with events
  static constexpr int kBins = 6;
  char* bws[kBins] = {nullptr};
  int64_t bws_cap[kBins] = {0};
  char* bjobs[kBins] = {nullptr};
  int64_t bjobs_cap[kBins] = {0};
  hipStream_t bstream[kBins] = {nullptr};
  hipEvent_t bev[kBins] = {nullptr};
  hipEvent_t fork_ev = nullptr;
  char* dhits = nullptr;
  int64_t dhits_cap = 0;
  double* dstats = nullptr;
  int64_t dstats_cap = 0;
  float* xbuf = nullptr;
  int64_t xbuf_cap = 0;
  int q_max_iter = 20;
  double q_tol = 0.01;
  int64_t lds_limit = 65536;  // dynamic LDS a workgroup may request
  bool poisoned = false;
  std::string err;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the last query launches
  std::vector<double> last_stats;           // per-job stats of the last query batch
  bool ev_valid = false;
};

namespace {

tk_status fail(tk_tree* t, tk_status st, const std::string& msg) {
  if (t) t->err = msg;
  else g_create_error = msg;
  return st;
}

tk_status fail_dev(tk_tree* t, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (t) {
    t->poisoned = true;
    t->err = m;
  } else {
    g_create_error = m;
  }
  return TK_EDEVICE;
}

#define TK_HIP(t, call)                                 \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return fail_dev(t, e_, #call); \
  } while (0)

tk_status ensure(tk_tree* t, char** buf, int64_t* cap, int64_t need, const char* what) {
  if (need <= *cap) return TK_OK;
  if (*buf) {
    TK_HIP(t, hipDeviceSynchronize());  // the buffer may be in use on any of the tree's streams
    TK_HIP(t, hipFree(*buf));
    *buf = nullptr;
    *cap = 0;
  }
  const int64_t sz = need + need / 4 + 4096;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, size_t(sz));
  if (e != hipSuccess) return fail_dev(t, e, what);
  *buf = static_cast<char*>(p);
  *cap = sz;
  return TK_OK;
}

int nu2_trailing_ones(int64_t b) {
  int n = 0;
  while (b & 1) {
    ++n;
    b >>= 1;
  }
  return n;
}

int eig_need(const tk::StitchLayout& lo, const StoreView& st, int s) {
  int n = lo.sk;
  for (int m = 1; m < st.p; ++m) {
    const int e = lo.sr[m] < st.D[m] ? lo.sr[m] : int(st.D[m]);
    if (e > n) n = e;
  }
  return n;
}

// Launch one bin of stitch jobs (all sharing n_lds) on stream `stream`,
// with workspace and job array `ws` / `djobs`; heaviest jobs first.  The
// hit array is already on the device.  Large bins are split into chunks
// bounded by workspace size (chunks of one bin run in order on its stream).
tk_status launch_bin(tk_tree* t, std::vector<Job>& jobs, const std::vector<Hit>& hits, int n_lds, int max_iter,
                     double tol, hipStream_t stream, char** ws, int64_t* ws_cap, char** djobs, int64_t* djobs_cap) {
  const int64_t nj = int64_t(jobs.size());
  if (nj == 0) return TK_OK;
  std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) {
    return a.s * a.L > b.s * b.L;  // longer ranges with more hits take longer
  });
  const size_t lds_bytes = size_t(tk::eig_doubles(n_lds)) * 8;
  std::vector<int64_t> off(static_cast<size_t>(nj) + 1, 0);
  for (int64_t i = 0; i < nj; ++i) {
    tk::StitchLayout lo;
    tk::stitch_layout(t->view, hits.data() + jobs[i].hit0, jobs[i].s, jobs[i].rq, n_lds, &lo);
    off[i + 1] = off[i] + lo.total;
  }
  int64_t i0 = 0;
  while (i0 < nj) {
    int64_t i1 = i0 + 1;
    while (i1 < nj && i1 - i0 < kMaxJobsPerLaunch && off[i1 + 1] - off[i0] <= kWsChunkBytes) ++i1;
    if (i0 > 0) TK_HIP(t, hipStreamSynchronize(stream));  // the buffers are reused by this chunk
    tk_status st = ensure(t, ws, ws_cap, off[i1] - off[i0] + 256, "workspace");
    if (st) return st;
    for (int64_t i = i0; i < i1; ++i) jobs[i].ws_off = off[i] - off[i0];
    st = ensure(t, djobs, djobs_cap, (i1 - i0) * int64_t(sizeof(Job)), "jobs");
    if (st) return st;
    TK_HIP(t, hipMemcpyAsync(*djobs, jobs.data() + i0, size_t(i1 - i0) * sizeof(Job), hipMemcpyHostToDevice,
                             stream));
    tk::StitchArgs a;
    a.st = t->dview;
    a.jobs = reinterpret_cast<const Job*>(*djobs);
    a.hits = reinterpret_cast<const Hit*>(t->dhits);
    a.ws = *ws;
    a.n_lds = n_lds;
    a.max_iter = max_iter;
    a.tol = tol;
    a.merge_max_iter = t->cfg.max_iter;
    a.merge_tol = t->cfg.tol;
    TK_HIP(t, tk::launch_stitch(a, int(i1 - i0), lds_bytes, n_lds > 48, stream));
    i0 = i1;
  }
  return TK_OK;
}

// Launch stitch jobs (queries or merges).  Jobs are binned by the size of
// their largest eigenproblem so that each launch sizes its LDS (and its
// wavefronts per job) for its own jobs: small problems keep many jobs per
// CU, large ones still run their eigensolves in LDS.  Bins run concurrently
// on their own streams and are joined back to the tree's stream, so a batch
// completes in about the time of its slowest bin.
tk_status run_stitch(tk_tree* t, std::vector<Job>& jobs, const std::vector<Hit>& hits, int max_iter,
                     double tol) {
  const int64_t nj = int64_t(jobs.size());
  if (nj == 0) return TK_OK;
  int lds_cap = 128;
  while (lds_cap > 8 && int64_t(tk::eig_doubles(lds_cap)) * 8 > t->lds_limit - int64_t(tk::stitch_static_lds()))
    lds_cap -= 8;
  int bins[tk_tree::kBins - 1] = {24, 32, 48, 64, 96};
  for (int& b : bins) b = b < lds_cap ? b : lds_cap;
  std::vector<std::vector<Job>> binned(tk_tree::kBins);
  for (int64_t i = 0; i < nj; ++i) {
    tk::StitchLayout lo;
    tk::stitch_layout(t->view, hits.data() + jobs[i].hit0, jobs[i].s, jobs[i].rq, 1 << 30, &lo);
    const int need = eig_need(lo, t->view, jobs[i].s);
    if (need > tk::EIG_MAXK_HOST) return fail(t, TK_EINVAL, "query needs an eigenproblem above 1024");
    int b = tk_tree::kBins - 1;
    for (int k = 0; k < tk_tree::kBins - 1; ++k)
      if (need <= bins[k]) {
        b = k;
        break;
      }
    binned[size_t(b)].push_back(jobs[i]);
  }
  tk_status st = ensure(t, &t->dhits, &t->dhits_cap, int64_t(hits.size() * sizeof(Hit)) + 64, "hits");
  if (st) return st;
  if (!hits.empty())
    TK_HIP(t, hipMemcpyAsync(t->dhits, hits.data(), hits.size() * sizeof(Hit), hipMemcpyHostToDevice,
                             t->stream));
  int nonempty = 0;
  for (auto& b : binned) nonempty += b.empty() ? 0 : 1;
  if (nonempty <= 1) {
    for (int b = 0; b < tk_tree::kBins; ++b)
      if (!binned[size_t(b)].empty())
        return launch_bin(t, binned[size_t(b)], hits, b < tk_tree::kBins - 1 ? bins[b] : lds_cap, max_iter, tol,
                          t->stream, &t->ws, &t->ws_cap, &t->djobs, &t->djobs_cap);
    return TK_OK;
  }
  if (!t->fork_ev) TK_HIP(t, hipEventCreateWithFlags(&t->fork_ev, hipEventDisableTiming));
  TK_HIP(t, hipEventRecord(t->fork_ev, t->stream));
  for (int b = 0; b < tk_tree::kBins; ++b) {
    if (binned[size_t(b)].empty()) continue;
    if (!t->bstream[b]) {
      TK_HIP(t, hipStreamCreateWithFlags(&t->bstream[b], hipStreamNonBlocking));
      TK_HIP(t, hipEventCreateWithFlags(&t->bev[b], hipEventDisableTiming));
    }
    TK_HIP(t, hipStreamWaitEvent(t->bstream[b], t->fork_ev, 0));
    st = launch_bin(t, binned[size_t(b)], hits, b < tk_tree::kBins - 1 ? bins[b] : lds_cap, max_iter, tol,
                    t->bstream[b], &t->bws[b], &t->bws_cap[b], &t->bjobs[b], &t->bjobs_cap[b]);
    if (st) return st;
    TK_HIP(t, hipEventRecord(t->bev[b], t->bstream[b]));
    TK_HIP(t, hipStreamWaitEvent(t->stream, t->bev[b], 0));
  }
  return TK_OK;
}

tk_status run_leaves(tk_tree* t, int64_t first_block, int64_t nb, const float* X) {
  if (nb <= 0) return TK_OK;
  tk::LeafLayout lo;
  tk::leaf_layout(t->view, 1 << 30, &lo);
  int cap = 128;
  while (cap > 8 && int64_t(tk::eig_doubles(cap)) * 8 > t->lds_limit - int64_t(tk::leaf_static_lds())) cap -= 8;
  const int n_lds = lo.neig < cap ? lo.neig : cap;
  tk::leaf_layout(t->view, n_lds, &lo);
  const size_t lds_bytes = size_t(tk::eig_doubles(n_lds)) * 8;
  const int64_t per = lo.total;
  int64_t chunk = kWsChunkBytes / (per > 0 ? per : 1);
  if (chunk < 1) chunk = 1;
  if (chunk > kMaxJobsPerLaunch) chunk = kMaxJobsPerLaunch;
  const int64_t block_elems = t->ell * t->slice_elems;
  for (int64_t i0 = 0; i0 < nb; i0 += chunk) {
    const int64_t n = (nb - i0) < chunk ? (nb - i0) : chunk;
    tk_status st = ensure(t, &t->ws, &t->ws_cap, n * per + 256, "workspace");
    if (st) return st;
    std::vector<LeafJob> jobs(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
      jobs[i].X = X + (i0 + i) * block_elems;
      jobs[i].block = first_block + i0 + i;
      jobs[i].stats = nullptr;
      jobs[i].ws_off = i * per;
    }
    st = ensure(t, &t->djobs, &t->djobs_cap, n * int64_t(sizeof(LeafJob)), "jobs");
    if (st) return st;
    TK_HIP(t, hipMemcpyAsync(t->djobs, jobs.data(), size_t(n) * sizeof(LeafJob), hipMemcpyHostToDevice,
                             t->stream));
    tk::LeafArgs a;
    a.st = t->dview;
    a.jobs = reinterpret_cast<const LeafJob*>(t->djobs);
    a.ws = t->ws;
    a.n_lds = n_lds;
    a.max_iter = t->cfg.max_iter;
    a.tol = t->cfg.tol;
    TK_HIP(t, tk::launch_leaf(a, int(n), lds_bytes, t->stream));
    TK_HIP(t, hipStreamSynchronize(t->stream));  // jobs/ws are reused by the next chunk
  }
  return TK_OK;
}

// Merge job for node (k, j): Stitch of its two children (Alg. "insert").
void merge_job(tk_tree* t, int k, int64_t j, std::vector<Job>& jobs, std::vector<Hit>& hits) {
  const StoreView& v = t->view;
  Job jb{};
  jb.kind = 1;
  jb.s = 2;
  jb.hit0 = int32_t(hits.size());
  jb.L = t->ell << k;
  for (int n = 0; n < t->p; ++n) jb.rq[n] = v.rk[k][n];
  jb.out_core = v.core[k] + j * v.core_elems[k];
  for (int n = 1; n < t->p; ++n) jb.out_fac[n] = v.fac[k][n] + j * tk::fac_elems(v, k, n);
  jb.out_fac[0] = v.plane[k] + (j << k) * t->ell * v.rk[k][0];
  jb.stats = nullptr;
  const int64_t half = t->ell << (k - 1);
  Hit h0{k - 1, 0, 2 * j, 0, half};
  Hit h1{k - 1, 0, 2 * j + 1, 0, half};
  hits.push_back(h0);
  hits.push_back(h1);
  jobs.push_back(jb);
}

// Leaves for blocks [Tb, Tb + nb) from device data, then every merge they
// complete, level by level.
tk_status commit_blocks(tk_tree* t, int64_t nb, const float* Xdev) {
  const int64_t b0 = t->Tb, b1 = t->Tb + nb;
  tk_status st = run_leaves(t, b0, nb, Xdev);
  if (st) return st;
  const int K = tk::root_level(b1);
  int64_t merges = 0;
  for (int k = 1; k <= K; ++k) {
    // nodes (k, j) with (j+1) 2^k in (b0, b1]
    const int64_t jlo = b0 >> k;
    const int64_t jhi = (b1 >> k) - 1;
    if (jhi < jlo) continue;
    std::vector<Job> jobs;
    std::vector<Hit> hits;
    for (int64_t j = jlo; j <= jhi; ++j) merge_job(t, k, j, jobs, hits);
    merges += int64_t(jobs.size());
    st = run_stitch(t, jobs, hits, t->cfg.max_iter, t->cfg.tol);
    if (st) return st;
  }
  t->Tb = b1;
  t->merges_total += merges;
  t->merges_last = nu2_trailing_ones(b1 - 1);
  return TK_OK;
}

bool range_ok(const tk_tree* t, int64_t ts, int64_t te) {
  return ts >= 0 && ts < te && te <= t->Tb * t->ell;
}

tk_status build_query_job(tk_tree* t, int64_t ts, int64_t te, const tk_result* res, std::vector<Job>& jobs,
                          std::vector<Hit>& hits) {
  if (!range_ok(t, ts, te)) return fail(t, TK_ERANGE, "query range outside [0, T_c) or empty");
  Hit buf[tk::MAXHITS];
  const int n = tk::recall(ts, te, t->Tb, t->ell, t->cfg.theta_num, t->cfg.theta_den, buf, tk::MAXHITS);
  if (n < 1 || n > tk::MAXHITS) return fail(t, TK_EINVAL, "hit set too large");
  Job jb{};
  jb.kind = 0;
  jb.s = n;
  jb.hit0 = int32_t(hits.size());
  jb.L = te - ts;
  tk::effective_ranks(t->p, te - ts, t->view.D, t->cfg.ranks, jb.rq);
  if (!res->core) return fail(t, TK_EINVAL, "null core buffer");
  for (int m = 0; m < t->p; ++m)
    if (!res->factor[m]) return fail(t, TK_EINVAL, "null factor buffer");
  jb.out_core = res->core;
  for (int m = 0; m < t->p; ++m) jb.out_fac[m] = res->factor[m];
  for (int i = 0; i < n; ++i) hits.push_back(buf[i]);
  jobs.push_back(jb);
  return TK_OK;
}

}  // namespace

extern "C" {

const char* tk_version(void) { return "0.1.0"; }

const char* tk_last_error(const tk_tree* t) { return t ? t->err.c_str() : g_create_error.c_str(); }

tk_status tk_create(const tk_config* cfg, void* hip_stream, tk_tree** out) {
  if (!cfg || !out) return fail(nullptr, TK_EINVAL, "null argument");
  *out = nullptr;
  const int p = cfg->p;
  if (p < 2 || p > tk::MAXP) return fail(nullptr, TK_EINVAL, "p must be in [2, 6]");
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
  if (cfg->prec != TK_F32) return fail(nullptr, TK_EINVAL, "only TK_F32 is available");
  if (cfg->capacity_T < cfg->leaf_len || cfg->capacity_T > (int64_t(1) << 40))
    return fail(nullptr, TK_EINVAL, "bad capacity_T");

  tk_tree* t = new tk_tree();
  t->cfg = *cfg;
  t->stream = static_cast<hipStream_t>(hip_stream);
  t->p = p;
  t->ell = cfg->leaf_len;
  t->slice_elems = slice;
  t->cap_blocks = cfg->capacity_T / cfg->leaf_len;
  t->nlev = tk::root_level(t->cap_blocks) + 1;
  t->q_max_iter = cfg->max_iter;
  t->q_tol = cfg->tol;
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
  (void)hipStreamSynchronize(t->stream);
  char* bufs[] = {t->store, t->ws, t->djobs, t->dhits};
  for (char* b : bufs)
    if (b) (void)hipFree(b);
  if (t->dview) (void)hipFree(t->dview);
  if (t->block_buf) (void)hipFree(t->block_buf);
  if (t->dstats) (void)hipFree(t->dstats);
  if (t->xbuf) (void)hipFree(t->xbuf);
  for (int b = 0; b < tk_tree::kBins; ++b) {
    if (t->bstream[b]) (void)hipStreamSynchronize(t->bstream[b]);
    if (t->bws[b]) (void)hipFree(t->bws[b]);
    if (t->bjobs[b]) (void)hipFree(t->bjobs[b]);
    if (t->bstream[b]) (void)hipStreamDestroy(t->bstream[b]);
    if (t->bev[b]) (void)hipEventDestroy(t->bev[b]);
  }
  if (t->fork_ev) (void)hipEventDestroy(t->fork_ev);
  if (t->ev0) (void)hipEventDestroy(t->ev0);
  if (t->ev1) (void)hipEventDestroy(t->ev1);
  delete t;
}

tk_status tk_append(tk_tree* t, const float* slice, int on_device) {
  if (!t || !slice) return fail(t, TK_EINVAL, "null argument");
  if (t->poisoned) return TK_EDEVICE;
  if (t->T >= t->cap_blocks * t->ell) return fail(t, TK_ENOMEM, "capacity_T reached");
  const int64_t row = t->T % t->ell;
  TK_HIP(t, hipMemcpyAsync(t->block_buf + row * t->slice_elems, slice, size_t(t->slice_elems) * 4,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, t->stream));
  t->T += 1;
  if (t->T % t->ell == 0) {
    tk_status st = commit_blocks(t, 1, t->block_buf);
    if (st) return st;
    TK_HIP(t, hipStreamSynchronize(t->stream));
  }
  return TK_OK;
}

tk_status tk_build(tk_tree* t, const float* X, int64_t T, int on_device) {
  if (!t || (!X && T > 0) || T < 0) return fail(t, TK_EINVAL, "bad argument");
  if (t->poisoned) return TK_EDEVICE;
  if (t->T + T > t->cap_blocks * t->ell) return fail(t, TK_ENOMEM, "capacity_T exceeded");
  int64_t done = 0;
  if (t->T % t->ell == 0) {
    const int64_t nb = T / t->ell;
    const int64_t block_elems = t->ell * t->slice_elems;
    if (nb > 0) {
      const float* Xd = X;
      if (!on_device) {
        tk_status st = ensure(t, reinterpret_cast<char**>(&t->xbuf), &t->xbuf_cap, nb * block_elems * 4, "staging");
        if (st) return st;
        TK_HIP(t, hipMemcpyAsync(t->xbuf, X, size_t(nb * block_elems) * 4, hipMemcpyHostToDevice, t->stream));
        Xd = t->xbuf;
      }
      tk_status st = commit_blocks(t, nb, Xd);
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
  if (!range_ok(t, ts, te)) return TK_ERANGE;
  Hit buf[tk::MAXHITS];
  const int m = tk::recall(ts, te, t->Tb, t->ell, t->cfg.theta_num, t->cfg.theta_den, buf, tk::MAXHITS);
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
  if (!range_ok(t, ts, te)) return TK_ERANGE;
  std::memset(out, 0, sizeof(*out));
  tk::effective_ranks(t->p, te - ts, t->view.D, t->cfg.ranks, out->ranks_eff);
  out->L = te - ts;
  out->core_elems = 1;
  for (int n = 0; n < t->p; ++n) out->core_elems *= out->ranks_eff[n];
  out->factor_elems[0] = out->L * out->ranks_eff[0];
  for (int n = 1; n < t->p; ++n) out->factor_elems[n] = t->view.D[n] * out->ranks_eff[n];
  Hit buf[tk::MAXHITS];
  out->n_hits = tk::recall(ts, te, t->Tb, t->ell, t->cfg.theta_num, t->cfg.theta_den, buf, tk::MAXHITS);
  return TK_OK;
}

tk_status tk_query_batch(tk_tree* t, int32_t n, const int64_t* ts, const int64_t* te, tk_result* res) {
  if (!t || n < 0 || (n > 0 && (!ts || !te || !res))) return fail(t, TK_EINVAL, "bad argument");
  if (t->poisoned) return TK_EDEVICE;
  std::vector<Job> jobs;
  std::vector<Hit> hits;
  jobs.reserve(size_t(n));
  for (int32_t i = 0; i < n; ++i) {
    tk_status st = build_query_job(t, ts[i], te[i], &res[i], jobs, hits);
    if (st) return st;
  }
  if (n == 0) return TK_OK;
  tk_status st = ensure(t, reinterpret_cast<char**>(&t->dstats), &t->dstats_cap,
                        int64_t(n) * tk::STAT_COUNT * 8, "stats");
  if (st) return st;
  for (int32_t i = 0; i < n; ++i) jobs[i].stats = t->dstats + tk::STAT_COUNT * int64_t(i);
  if (!t->ev0) {
    TK_HIP(t, hipEventCreate(&t->ev0));
    TK_HIP(t, hipEventCreate(&t->ev1));
  }
  t->ev_valid = false;
  TK_HIP(t, hipEventRecord(t->ev0, t->stream));
  st = run_stitch(t, jobs, hits, t->q_max_iter, t->q_tol);
  if (st) return st;
  TK_HIP(t, hipEventRecord(t->ev1, t->stream));
  t->ev_valid = true;
  std::vector<double>& hs = t->last_stats;
  hs.assign(size_t(n) * tk::STAT_COUNT, 0.0);
  TK_HIP(t, hipMemcpyAsync(hs.data(), t->dstats, hs.size() * 8, hipMemcpyDeviceToHost, t->stream));
  TK_HIP(t, hipStreamSynchronize(t->stream));
  for (int32_t i = 0; i < n; ++i) {
    const double* s = hs.data() + tk::STAT_COUNT * size_t(i);
    for (int m = 0; m < tk::MAXP; ++m) res[i].ranks_eff[m] = m < t->p ? jobs[i].rq[m] : 0;
    res[i].fit = s[tk::STAT_FIT];
    res[i].err_model = s[tk::STAT_ERR];
    res[i].norm_ytilde = s[tk::STAT_NORM];
    res[i].sweeps = int32_t(s[tk::STAT_SWEEPS]);
    res[i].converged = int32_t(s[tk::STAT_CONV]);
    res[i].n_hits = jobs[i].s;
  }
  return TK_OK;
}

tk_status tk_query(tk_tree* t, int64_t ts, int64_t te, tk_result* res) {
  return tk_query_batch(t, 1, &ts, &te, res);
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
  for (int k = 0; k < tk::STAT_NPHASE + 4; ++k)
    phase_us[k] = t->last_stats[size_t(i) * tk::STAT_COUNT + tk::STAT_PHASE + k];
  return TK_OK;
}

tk_status tk_set_query_iters(tk_tree* t, int32_t max_iter, double tol) {
  if (!t || max_iter < 1 || !(tol >= 0.0)) return TK_EINVAL;
  t->q_max_iter = max_iter;
  t->q_tol = tol;
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
  if (t->poisoned) return TK_EDEVICE;
  t->T = T;
  t->Tb = T / t->ell;
  t->merges_total = 0;
  t->merges_last = 0;
  return TK_OK;
}

tk_status tk_load_node(tk_tree* t, int32_t level, int64_t index, const float* core,
                       const float* const* factor) {
  if (!t || !core || !factor || level < 0 || level >= t->nlev || index < 0) return TK_EINVAL;
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
