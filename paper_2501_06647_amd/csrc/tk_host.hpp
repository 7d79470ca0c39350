// Host-side state of a tree and the planning/launch helpers shared by the
// synchronous calls (tk_capi.hip), prepared batches (tk_batch.hip) and the
// serving engine (tk_serve.hip).
#pragma once

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "tk_internal.hpp"
#include "tk_tune_search.hpp"
#include "tucket.h"

namespace tk {

constexpr int kMaxRank = 32;
constexpr int kMaxGroups = 7;                          // LDS bins of a stitch launch
// Streams a batch's groups are spread over (the process has four hardware
// queues); groups beyond this many share streams, lighter groups after
// heavier ones.
constexpr int kForkStreams = 4;
constexpr int64_t kMaxJobsPerLaunch = 1 << 16;
constexpr int64_t kWsChunkBytes = int64_t(4) << 30;    // workspace per launch chunk
constexpr size_t kLdsBytes = 160 * 1024;               // LDS per CU on gfx950

struct DevBuf {
  char* p = nullptr;
  int64_t cap = 0;
  bool fixed = false;  // memory owned elsewhere (the no-allocation scratch): never reallocated or freed
};

// Launch tuning of the stitch kernel (tk_tuning).
struct Tuning {
  int wide_threshold = 48;  // jobs whose largest eigenproblem exceeds this use wide workgroups
  int wide_threads = 256;
  int persistent = 0;       // grid sized to residency; workgroups pull jobs from a queue
  int graph = 1;            // prepared batches replay a captured HIP graph
  int coarse = 0;           // 1: LDS bins {32, wide_threshold, 96} instead of {24, 32, 48, 64, 96, threshold}
  int lds_n = 0;            // largest eigenproblem held in LDS (0: as large as fits); >= wide_threshold
  int basis_pct = 75;       // mode n uses the span basis when 100 sr_n < basis_pct D_n
  int rest_threads = 0;     // block size of the bin above the LDS cap (0: wide_threads)
  int wide_core = 0;        // cores above this many elements run wide (0: off)
};

// Stitch jobs that run in one launch: same dynamic LDS (n_lds) and block size.
struct Group {
  int bin = 0;     // index of the LDS bin (stable across calls: selects buffers)
  int slot = 0;    // fork stream of the group
  int n_lds = 0;
  int lds_doubles = 0;  // dynamic LDS: the n_lds eigen buffer, or the vector part of the largest job's
  int threads = 64;
  std::vector<Job> jobs;
  int64_t ws_total = 0;
};

// Dynamic LDS (doubles) of a launch whose eigenproblems up to n_lds run in
// LDS and whose largest has size need.
int64_t group_lds_doubles(int n_lds, int need);

// A stitch batch split into groups, each sorted heaviest first, with
// workspace offsets relative to the group's buffer.
struct Plan {
  std::vector<Hit> hits;
  std::vector<Group> groups;
  int64_t n_jobs = 0;
  int basis_pct = 75;  // the tuning the plan was made under
};

// A stream with the device buffers of the stitch work issued on it.  Groups
// of one batch run on the lane's group streams when forked, else one after
// the other on the lane's stream.
struct Lane {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevBuf hits, stats, queue;
  DevBuf ws[kMaxGroups], jobs[kMaxGroups], trims[kMaxGroups];
  DevBuf leaf_ws, leaf_jobs, xbuf;
  DevBuf sx[6];  // streaming Tucker-ALS: projections, partials, Y, U^(1), small buffers, solver
  hipStream_t gstream[kMaxGroups] = {};
  hipEvent_t gev[kMaxGroups] = {};
  hipEvent_t fork_ev = nullptr;
};

struct Server;  // tk_serve.hip

}  // namespace tk

struct tk_tree {
  tk_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 256;
  int p = 0;
  int64_t ell = 1;
  int64_t cap_blocks = 0;
  int nlev = 0;
  tk::StoreView view{};
  tk::StoreView* dview = nullptr;
  char* store = nullptr;
  int64_t store_bytes = 0;
  float* block_buf = nullptr;
  int64_t slice_elems = 0;
  int64_t T = 0;
  int64_t Tb = 0;
  int64_t merges_total = 0;
  int64_t merges_last = 0;
  tk::Lane main;  // the tree's stream: synchronous calls
  int q_max_iter = 20;
  double q_tol = 0.01;
  int q_prec = TK_F32;  // arithmetic of query stitches (merges follow cfg.prec)
  int32_t q_ranks[TK_MAX_MODES] = {};  // output ranks of queries (0: cfg.ranks)
  int q_level = -1;                    // queries' hit sets: Alg. recall (-1) or fixed blocks of this level
  int64_t prov_T = -1;                 // T at which the provisional leaf in slot Tb was computed (-1: none)
  int64_t tail_rows = 0;               // leading rows of block_buf holding the incomplete block's slices
  tk::DevBuf prov_out;                 // its compact decomposition
  int64_t lds_limit = 65536;  // dynamic + static LDS a workgroup may use
  tk::Tuning tuning;
  tk::TuneLimits tune_limits;  // time budget, abandonment cap and progress output of tk_autotune
  std::atomic<bool> poisoned{false};
  // last error text; written by the caller's threads and the serving
  // engine's thread, so always under err_mu (set_error / tk_last_error)
  std::string err;
  mutable std::mutex err_mu;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the last query launches
  std::vector<double> last_stats;           // per-job stats of the last query batch
  bool ev_valid = false;
  tk::Server* server = nullptr;             // non-null while serving
};

namespace tk {

tk_status fail(tk_tree* t, tk_status st, const std::string& msg);
// Record msg as the tree's last error (thread-safe).
void set_error(tk_tree* t, const std::string& msg);
// Error text for a stitch job's nonzero STAT_STATUS: 1 the kernel's Recall
// did not reproduce the planned hit set, 2 the workspace plan was too small,
// 3 the launch's LDS could not hold the job's eigen vectors or its kernel
// instantiation holds fewer modes than the tree (the job did nothing in
// cases 2 and 3).
std::string job_status_msg(double status);
tk_status fail_dev(tk_tree* t, hipError_t e, const char* what);

#define TK_HIP(t, call)                                         \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return ::tk::fail_dev(t, e_, #call); \
  } while (0)

// Grow b to at least need bytes (waits for the device before freeing).
tk_status ensure(tk_tree* t, DevBuf* b, int64_t need, const char* what);
void release(DevBuf* b);
void lane_destroy(Lane* l);

// Largest eigenproblem of a stitch job (its LDS bin).
int eig_need(const tk_tree* t, const StitchLayout& lo);

// Recall plus effective ranks of a query at snapshot Tb: one job (hits
// appended to `hits`).  Output buffers from res (may be null when
// check_outputs is false).
tk_status make_query_job(tk_tree* t, int64_t ts, int64_t te, int64_t Tb, const tk_result* res, bool check_outputs,
                         std::vector<Job>& jobs, std::vector<Hit>& hits, bool tail_ok = false);
// The hits of [ts, te) at snapshot Tb; with tail_ok (Tb the tree's) a range
// may end in the incomplete block, whose provisional leaf in slot Tb is the
// last hit (*tail set).  Returns the number of hits needed, or -1 if the
// range is outside what the call may reach.
int plan_query_hits(const tk_tree* t, int64_t ts, int64_t te, int64_t Tb, bool tail_ok, Hit* out, int cap,
                    bool* tail);
// Tucker-ALS of the incomplete block into slot Tb, zero-padded to the slot's
// shapes (once per horizon T; tk_tail.hip).
tk_status provisional_leaf(tk_tree* t);
// Merge job for node (k, j): Stitch of its two children (Alg. "insert").
void make_merge_job(tk_tree* t, int k, int64_t j, std::vector<Job>& jobs, std::vector<Hit>& hits);

// Group jobs by LDS bin under the tree's tuning, sort each group heaviest
// first and lay out its workspace.
// Group and order stitch jobs (see tk_capi.hip).  With pretrim (prepared
// batches), query jobs whose partial hits hold at least kPretrimRows rows
// get their trims' row Grams from the trim pass (which the launcher of the
// plan then runs, trim_chunks_of + launch_trim, before the group's stitch
// launch); its chunked sums round differently from the stitch kernel's own,
// so those queries may differ from tk_query in the last bits.
tk_status plan_stitch(tk_tree* t, std::vector<Job>& jobs, std::vector<Hit>& hits, Plan* plan, bool pretrim = false);
constexpr int64_t kPretrimRows = 2048;
constexpr int kMergeThreads = 128;  // least threads of a merge job (append commits, builds)
// The trim-pass chunks of jobs [i0, i1) of a group whose workspace chunk
// starts at job i0's offset and lives at ws_base.
void trim_chunks_of(const tk_tree* t, const Plan& plan, const Group& gr, int64_t i0, int64_t i1, char* ws_base,
                    std::vector<TrimChunk>& out);

// Issue a plan on a lane: hits and jobs uploaded, groups launched (forked
// onto group streams when fork is set and there are several groups), the
// lane's stream joined.  Groups too large for one launch are chunked, with a
// host wait between chunks.
tk_status run_plan(tk_tree* t, Lane* lane, Plan& plan, int max_iter, double tol, bool fork);

// Leaves for blocks [Tb, Tb + nb) from device data, then every merge they
// complete, level by level, on the lane.  Updates Tb and the merge counts.
// Commit nb leaf blocks (leaves, then merges level by level) on the lane's
// stream.  With lev_ev, event lev_ev[k] is recorded once the nodes of level
// k are written, for k <= the new root level (and < n_ev).
tk_status commit_blocks(tk_tree* t, Lane* lane, int64_t nb, const float* Xdev, hipEvent_t* lev_ev = nullptr,
                        int n_ev = 0);

StitchArgs stitch_args(tk_tree* t, int max_iter, double tol);
// Output ranks of a query of length len (tk_set_query_ranks, clipped).
void query_ranks(const tk_tree* t, int64_t len, int32_t* out);
// The hit set a query of the tree uses (tk_set_query_recall): Alg. recall or
// fixed blocks; returns the number of hits needed.
int query_hits(const tk_tree* t, int64_t ts, int64_t te, int64_t Tb, Hit* out, int cap);
int lds_cap(const tk_tree* t);

}  // namespace tk
