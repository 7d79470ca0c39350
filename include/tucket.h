/*
 * tucket.h -- C ABI of the MI355X TUCKET range-query engine.
 *
 * Operations follow the paper's problem statement (Qiu et al., PVLDB 17(13),
 * 2024, Sec. 3): a tensor stream X in R^{* x D_2 x ... x D_p} whose first mode
 * is time receives slices X_T (stream update), and a range query [t_s, t_e)
 * returns a Tucker decomposition of X[t_s:t_e): a core G of size
 * r_1 x ... x r_p and factors U^(1) ((t_e - t_s) x r_1), U^(n) (D_n x r_n).
 * The data structure is the stream segment tree of Sec. 4.2 (built by
 * Alg. "append"/"insert", Sec. 6.2); queries run Alg. "recall" (Sec. 5.1)
 * and Alg. "stitch" (Sec. 5.2) on the device.
 *
 * Conventions
 *   - Tensors are C-order (row-major), time first (App. A: vec is C-order,
 *     mat_n rows run over mode n).  Factors are [rows][columns] row-major.
 *   - Modes are numbered 0..p-1 in arrays; index 0 is the temporal mode.
 *   - Every floating-point buffer crossing the ABI is IEEE binary32.
 *   - "device" pointers are HIP device allocations on the device that was
 *     current when the tree was created; "host" pointers are ordinary memory.
 *   - Leaves hold blocks of leaf_len slices; only whole blocks are committed,
 *     so a query needs 0 <= t_s < t_e <= T_c = leaf_len * floor(T / leaf_len).
 *   - Output ranks are the effective ranks of the range: r_1 <= length,
 *     r_n <= D_n, and r_n <= prod_{m != n} r_m (tk_query_shape reports them).
 *
 * Errors: every call returns a tk_status and never aborts.  Argument checks
 * happen before any device work.  A failed device call returns TK_EDEVICE
 * and poisons the tree (later calls return TK_EDEVICE); tk_last_error()
 * gives the message.
 */
#ifndef TUCKET_H
#define TUCKET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TK_MAX_MODES 8

typedef enum {
  TK_OK = 0,
  TK_EINVAL = 1,  /* bad argument (dims, ranks, null pointer, ...)          */
  TK_ERANGE = 2,  /* query range outside [0, T_c), or t_s >= t_e              */
  TK_ENOMEM = 3,  /* capacity or memory budget exceeded                      */
  TK_EDEVICE = 4, /* a HIP call failed; the tree is poisoned                 */
  TK_EBUSY = 5    /* serving: queue full, or a call that the server excludes  */
} tk_status;

/* Arithmetic of the stitch's ALS contractions (TTM chains, the mode
 * unfoldings Z^(n), the core update) and of their Grams, on the matrix
 * cores.  Eigensolves, orthonormalisation, trims, the final core and the
 * error norms are FP64 in both modes; stored data and outputs are FP32. */
typedef enum {
  TK_F32 = 1,  /* FP32 operands, FP32 accumulation (Grams: FP64 sums)      */
  TK_BF16 = 2  /* BF16 operands (round to nearest even), FP32 accumulation */
} tk_prec;

typedef struct tk_tree tk_tree;

/* Tree configuration.  Hyperparameter defaults of Sec. 8.1: max_iter 20,
 * tol 0.01, theta 0.7. */
typedef struct {
  int32_t p;                      /* number of modes, 2..7 (time included)   */
  int64_t dims[TK_MAX_MODES];     /* dims[1..p-1] = D_2..D_p; dims[0] unused */
  int32_t ranks[TK_MAX_MODES];    /* target ranks r_1..r_p                   */
  int32_t leaf_len;               /* slices per leaf block, >= 1             */
  int32_t theta_num, theta_den;   /* pruning threshold theta = num/den       */
  int32_t max_iter;               /* ALS sweep cap (>= 1)                    */
  double tol;                     /* stop when |fit_k - fit_{k-1}| < tol     */
  int32_t prec;                   /* tk_prec of merges and (initially) queries */
  int64_t capacity_T;             /* maximum number of slices                */
  int64_t mem_budget_bytes;       /* device bytes the tree may use; 0 = any  */
} tk_config;

/* One member of a pruned hit set (Alg. "recall"). */
typedef struct {
  int32_t level;     /* node covers leaf blocks [index 2^level, (index+1) 2^level) */
  int32_t partial;   /* 1 if the node is only partly inside the query           */
  int64_t index;
  int64_t node_id;   /* 1-based creation order (numbering of Fig. "illust")     */
  int64_t sigma;     /* node range [sigma, tau) in slices                       */
  int64_t tau;
  int64_t lo;        /* clipped range [lo, hi) = [t_s, t_e) & [sigma, tau)      */
  int64_t hi;
} tk_hit;

/* Shape of a query's output. */
typedef struct {
  int32_t ranks_eff[TK_MAX_MODES]; /* effective output ranks                   */
  int64_t L;                       /* t_e - t_s                                */
  int64_t core_elems;              /* prod of ranks_eff                        */
  int64_t factor_elems[TK_MAX_MODES]; /* [0] = L r_1; [n] = D_n r_n            */
  int32_t n_hits;
  int64_t ws_bytes;                /* device workspace of the query, at most   */
} tk_shape;

/* A query result.  core and factor[0..p-1] are caller-owned DEVICE buffers of
 * at least the sizes tk_query_shape reports (float elements); the call
 * fills the other fields. */
typedef struct {
  float* core;
  float* factor[TK_MAX_MODES];
  int32_t ranks_eff[TK_MAX_MODES];
  int32_t sweeps;      /* ALS sweeps run (0: the range is one stored node)     */
  int32_t converged;   /* 1 if the fit-change rule stopped the loop            */
  int32_t n_hits;
  double fit;          /* 1 - |Y~ - Y^| / |Y~|                                 */
  double err_model;    /* |Y~ - Y^| / |Y~|, Y~ = concatenated hit pieces       */
  double norm_ytilde;  /* |Y~|_F                                               */
} tk_result;

typedef struct {
  int64_t T;             /* slices appended                                   */
  int64_t T_committed;   /* slices in complete leaf blocks (queryable)        */
  int64_t blocks;        /* complete leaf blocks                              */
  int64_t nodes;         /* nodes created, placeholders included              */
  int64_t merges_total;  /* stitches run by appends                           */
  int64_t merges_last;   /* stitches run by the last completed block          */
  int64_t store_bytes;   /* device bytes held by the node store               */
  int32_t height;        /* tree height (Thm. "height-T")                     */
} tk_stats;

/* Create an empty tree (the problem statement, Sec. 3: dimensions, target
 * ranks, leaf length, theta, sweep cap and tolerance, capacity).
 * hip_stream: a hipStream_t (NULL = default stream);
 * all device work of the tree is ordered on it.  The node store for
 * capacity_T slices is allocated here.  *out is owned by the caller and
 * released with tk_destroy. */
tk_status tk_create(const tk_config* cfg, void* hip_stream, tk_tree** out);
void tk_destroy(tk_tree* t);
const char* tk_last_error(const tk_tree* t);

/* Stream update (Sec. 3; Alg. "append"): one slice of D_2 x ... x D_p FP32
 * values, on the host (copied before return) or on the device (read in
 * stream order).  When a leaf block completes, the leaf Tucker decomposition
 * (Tucker-ALS, Sec. 2) and the stitches of Alg. "insert" run on the device. */
tk_status tk_append(tk_tree* t, const float* slice, int on_device);

/* Build = T successive stream updates (Sec. 3; Alg. "append" applied to
 * slices 0..T-1, Sec. 6.2): X holds T x D_2 x ... x D_p FP32 values, C-order,
 * on the host or (on_device) the device.  Executed level by level: all new
 * leaves in one launch, then each tree level's merges (Alg. "insert"); the
 * stored nodes are the same as T calls of tk_append.  TK_ENOMEM past
 * capacity_T; a host X is copied before return. */
tk_status tk_build(tk_tree* t, const float* X, int64_t T, int on_device);

/* Pruned hit set of [t_s, t_e) in time order (host-side, bit-exact
 * integer Alg. "recall", or the fixed-block set if tk_set_query_recall
 * chose one).  Writes at most cap hits; *n = hits needed. */
tk_status tk_hitset(const tk_tree* t, int64_t ts, int64_t te, tk_hit* out,
                    int32_t cap, int32_t* n);

/* Output shape of a range query (Sec. 3: the core is r_1 x ... x r_p,
 * U^(1) is (t_e - t_s) x r_1, U^(n) is D_n x r_n), with the ranks clipped to
 * what the range admits, the size of its pruned hit set (Alg. "recall") and
 * its device workspace; ranges as tk_query accepts them (TK_ERANGE
 * otherwise).  Host-only, no device work. */
tk_status tk_query_shape(const tk_tree* t, int64_t ts, int64_t te, tk_shape* out);

/* Range query (Sec. 6.1): Recall, partial-hit trims (Eq. "partial-tucker")
 * and Stitch, one device launch.  Blocks until the result is written.  The
 * range may end past the last complete block (t_e <= T, leaf_len > 1):
 * the incomplete block's slices then get a provisional leaf (its Tucker-ALS
 * at the node ranks clipped to their count, computed once per horizon T in
 * the next leaf slot and replaced by the real leaf when the block
 * completes), stitched as a partial hit.  Only slices appended with
 * tk_append / tk_build (or kept by tk_serve_stop) count; after
 * tk_restore_begin the range ends at the last complete block.  Prepared
 * batches and served queries end there too (TK_ERANGE). */
tk_status tk_query(tk_tree* t, int64_t ts, int64_t te, tk_result* res);

/* tk_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same Recall, trims and Stitch kernels, with every device buffer the call
 * needs (hit list, queue counters, statistics, job descriptor, workspace)
 * taken from one fixed scratch array of 32 MiB per device, held by the
 * library from its load until the process ends; nothing is allocated or
 * freed.  The caller passes the output buffers as for tk_query.  The range
 * must end at or before the last complete block (else TK_ERANGE); a query
 * whose workspace exceeds the scratch returns TK_ENOMEM before any device
 * work.  Blocks until the result is written.  Every call on one device
 * shares that device's scratch (it keeps the last call's contents):
 * concurrent calls on one device, from any tree or thread, race. */
tk_status tk_query_noalloc(tk_tree* t, int64_t ts, int64_t te, tk_result* res);

/* n range queries stitched in one device launch (one workgroup per query).
 * Each query's result is identical to what tk_query returns for it. */
tk_status tk_query_batch(tk_tree* t, int32_t n, const int64_t* ts, const int64_t* te,
                         tk_result* res);

/* Device time, in milliseconds, of the stitch launches issued by the last
 * tk_query / tk_query_batch call, measured with HIP events recorded on the
 * tree's stream around those launches (instrumentation for benchmarks). */
tk_status tk_last_query_kernel_ms(const tk_tree* t, double* ms);

/* Device time of query i of the last tk_query_batch call split into its
 * eight phases, in microseconds (a 100 MHz wall clock read by the query's
 * workgroup): partial-hit trims, factor-span bases, HOSVD initialisation,
 * temporal-mode contractions and Gram, temporal-mode eigensolve, other
 * modes' contractions and Grams (with the core update), their eigensolves,
 * and writing the result; then four eigensolver counters: calls, bisection
 * steps, microseconds computing eigenvalues (tridiagonalisation and
 * bisection), microseconds computing eigenvectors; then the query's start
 * and end on the device clock in microseconds; then the number of
 * eigensolves whose vectors needed the Gram-Schmidt fallback; then the
 * microseconds of the eigenvalue time spent tridiagonalising and of the
 * eigenvector time spent in inverse iteration (those counters cover the
 * full solver only); then four for the sweeps' warm-started eigensolves
 * (subspace iteration from the previous sweep's vectors, kept when a
 * certificate shows it found the leading subspace): accepted, refused (the
 * full solver ran after them), their iteration steps, their microseconds;
 * then the part of those microseconds spent in their Rayleigh-Ritz step.
 * phase_us has 22 entries. */
tk_status tk_last_query_profile(const tk_tree* t, int32_t i, double* phase_us);

/* Override the ALS sweep cap and tolerance for later queries (not merges). */
tk_status tk_set_query_iters(tk_tree* t, int32_t max_iter, double tol);

/* Arithmetic (tk_prec) of later queries; merges keep cfg.prec.  Lets one
 * node store answer the same queries in FP32 and in BF16. */
tk_status tk_set_query_prec(tk_tree* t, int32_t prec);

/* Output ranks r_1..r_p of later queries (Alg. "stitch" takes the target
 * ranks as an input): ranks[n] in [1, cfg.ranks[n]], clipped like the node
 * ranks to what each range admits (tk_query_shape reports them); NULL
 * restores cfg.ranks.  A range equal to one stored node is returned verbatim
 * only at the node's own ranks, else it is stitched from that node alone.
 * Merges keep cfg.ranks.  TK_EINVAL if out of range, TK_EBUSY while
 * serving. */
tk_status tk_set_query_ranks(tk_tree* t, const int32_t* ranks);

/* Tucker-ALS from scratch on raw ranges (the accuracy reference and naive
 * baseline of the paper's comparisons): X[i] is a DEVICE array of L[i]
 * slices (L[i] x D_2 x ... x D_p floats, C order), res[i] sized by
 * tk_query_shape for a range of that length (same output ranks as a query,
 * tk_set_query_ranks included).  HOSVD init of U^(2..p), sweeps from the
 * temporal mode, the query sweep cap and tolerance, fields filled as for a
 * query (err_model against X, n_hits 0).  One workgroup per range, all
 * ranges in one launch (chunked by workspace); synchronous on the tree's
 * stream.  TK_EINVAL for null buffers or L outside [1, 2^30]. */
tk_status tk_raw_tucker(tk_tree* t, int32_t n, const float* const* X, const int64_t* L, tk_result* res);

/* Tucker-ALS from scratch on one long raw range with many workgroups: the
 * same iteration as tk_raw_tucker (Sec. 2's Tucker-ALS, HOSVD init of
 * U^(2..p), sweeps from the temporal mode, the query sweep cap, tolerance and
 * output ranks), with each pass over the range split into spans of
 * consecutive slices, one workgroup per span (at most 512), and the spans'
 * partial Grams and mode products summed in a fixed order.  Every pass reads
 * the range once: p passes per sweep, bound by HBM.  X is a DEVICE array of
 * L slices (L x D_2 x ... x D_p floats, C order) that must stay valid until
 * the call returns; res is sized by tk_query_shape for length L (core and
 * factors caller-owned device buffers, written in FP32; the factors also
 * serve as the passes' FP32 operands).  Synchronous on the tree's stream; the
 * library keeps its working buffers (about L (R_1 + 2 r_1) 8 bytes plus
 * 512 spans' partials, R_1 the product of the non-temporal output ranks)
 * until tk_destroy.  A temporal factor of rank below r_1 (zero singular
 * values) keeps zero columns instead of being completed to an orthonormal
 * basis.  TK_EINVAL for null buffers, L outside [1, 2^31), a slice dimension
 * above 1024 or R_1 above 1024. */
tk_status tk_raw_tucker_stream(tk_tree* t, const float* X, int64_t L, tk_result* res);

/* Hit sets of later queries: level -1 (default) is Alg. "recall" with the
 * tree's theta; level >= 0 the fixed-block variant of the paper's
 * efficiency-accuracy comparison: every complete node of that level
 * (blocks of leaf_len 2^level slices) overlapping the range, clipped, and
 * Alg. "recall" on the part past the last complete block.  The stitch is
 * the same; tk_hitset reports the set in use.  TK_EINVAL for a level the
 * tree does not have, TK_EBUSY while serving. */
tk_status tk_set_query_recall(tk_tree* t, int32_t level);

/* Counters of the tree (tk_stats above): slices appended, the committed
 * horizon, blocks, nodes, height, node-store bytes, and the merges of
 * Alg. "insert" in total and for the last block (one per block amortized,
 * Prop. "time_complexity_appending").  Host-only; TK_EINVAL for null
 * arguments. */
tk_status tk_stats_get(const tk_tree* t, tk_stats* out);

/* Node store access (checkpoint/restore and tests).  A node (level, index)
 * is complete once (index+1) 2^level <= blocks.  Buffers are HOST float
 * arrays: core of prod(r_eff(level)) elements, factor[0] of
 * (leaf_len 2^level) x r_1 elements, factor[n] of D_n x r_n elements, with
 * r_eff the effective ranks of a range of length leaf_len 2^level. */
tk_status tk_node_ranks(const tk_tree* t, int32_t level, int32_t* ranks_eff);
tk_status tk_read_node(tk_tree* t, int32_t level, int64_t index, float* core,
                       float* const* factor);
/* Set the committed horizon to T slices without computing anything, then
 * load complete nodes with tk_load_node.  Queries are valid once every node
 * they touch is loaded.  T must be a multiple of leaf_len (a whole number of
 * leaf blocks; the slices of an incomplete block belong to no node, so a
 * horizon inside a block could not be continued by later appends): else
 * TK_EINVAL, before any device work. */
tk_status tk_restore_begin(tk_tree* t, int64_t T);
tk_status tk_load_node(tk_tree* t, int32_t level, int64_t index, const float* core,
                       const float* const* factor);

/* ---------------------------------------------------------------------------
 * Launch tuning, prepared batches and the autotuner.
 *
 * Stitch jobs are grouped into LDS bins by the size of their largest
 * eigenproblem.  Jobs up to wide_threshold run one wavefront per workgroup;
 * larger ones run wide_threads threads.  With persistent = 1 a launch has at
 * most as many workgroups as the device holds at once and each workgroup
 * takes jobs from a queue, heaviest first.  A query's mode n works in an
 * orthonormal basis of its pieces' mode-n factor spans (sr_n concatenated
 * columns of length D_n) when 100 sr_n < basis_pct D_n, else in the D_n
 * coordinates.  A job's result depends on the tuning only through
 * wide_threshold, wide_threads (reduction orders) and basis_pct (the
 * coordinates: equal in exact arithmetic).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t wide_threshold; /* 16..1024, default 48                              */
  int32_t wide_threads;   /* 128 or 256, default 256                           */
  int32_t persistent;     /* 0 or 1, default 0                                 */
  int32_t graph;          /* 1: prepared batches replay a captured HIP graph   */
  int32_t coarse;         /* 1: LDS bins {32, wide_threshold, 96} (fewer      */
                          /* launches), 0: {24, 32, 48, 64, 96, threshold}    */
  int32_t lds_n;          /* largest eigenproblem kept in LDS, 0 = as large   */
                          /* as fits; else >= wide_threshold (larger ones     */
                          /* run in HBM, more jobs share a CU)                */
  int32_t basis_pct;      /* 1..100, default 75 (see above)                   */
  int32_t rest_threads;   /* block size of the bin above the LDS cap (its     */
                          /* matrices in HBM): 128, 256, or 0 = wide_threads  */
  int32_t wide_core;      /* jobs whose core has more elements run in wide    */
                          /* workgroups whatever their eigenproblems (0: off) */
} tk_tuning;

tk_status tk_get_tuning(const tk_tree* t, tk_tuning* out);
tk_status tk_set_tuning(tk_tree* t, const tk_tuning* in);   /* TK_EINVAL if out of range */

/* A prepared batch: n range queries planned once at the current committed
 * horizon T_c (the snapshot), job descriptors resident on the device, and
 * (tuning.graph = 1) the launches captured in a HIP graph: per LDS bin a
 * trim pass that sums the row Grams of long partial hits (queries whose
 * partial hits hold 2048 rows or more) over chunks of 1024 rows with every
 * thread of many workgroups, then one fused stitch kernel that runs Recall
 * (Alg. "recall") on each query's range and snapshot, the partial-hit trims
 * (Eq. "partial-tucker") and the Stitch (Alg. "stitch").  res[0..n-1] are
 * caller-owned and must stay valid until tk_batch_destroy; their
 * core/factor buffers are device buffers sized by tk_query_shape.  Results
 * equal those of tk_query_batch under the same tuning, except for queries
 * with such long partial hits, whose chunked Gram sums round differently
 * (last bits; within the parity tolerances).  Later appends do not change
 * what a batch computes (completed nodes are immutable). */
typedef struct tk_batch tk_batch;
tk_status tk_batch_create(tk_tree* t, int32_t n, const int64_t* ts, const int64_t* te,
                          tk_result* res, tk_batch** out);
/* Enqueue one execution on the tree's stream and return (no host wait). */
tk_status tk_batch_run(tk_batch* b);
/* Wait for the last execution and fill res[i]'s scalar fields. */
tk_status tk_batch_wait(tk_batch* b);
/* Device time of the last execution (HIP events on the tree's stream). */
tk_status tk_batch_kernel_ms(const tk_batch* b, double* ms);
/* Per-query phase times of the last execution (as tk_last_query_profile). */
tk_status tk_batch_profile(const tk_batch* b, int32_t i, double* phase_us);
/* The hit set query i's kernel computed on the device (after a run). */
tk_status tk_batch_hits(const tk_batch* b, int32_t i, tk_hit* out, int32_t cap, int32_t* n);
void tk_batch_destroy(tk_batch* b);

/* Limits of tk_autotune's search (defaults: 60 s, cap 3, no progress).
 * budget_s: no new candidate starts once this many seconds have passed
 * since the search began (0: no limit); the best so far is kept and the
 * re-timing stage is skipped.  cap: a candidate whose warm-up execution
 * already takes more than cap times the best mean so far is not timed
 * further (0 or 1: never abandon).  progress: one line per candidate on
 * stderr.  TK_EINVAL for negative or NaN limits. */
tk_status tk_set_autotune_limits(tk_tree* t, double budget_s, double cap, int32_t progress);

/* Time every candidate tuning (wide_threshold in {32, 48, 64, 96} x
 * wide_threads in {128, 256} x lds_n in {32, 48, 64, 96, 0} (>= the threshold) x
 * persistent in {0, 1} x coarse in {0, 1} at basis_pct 75, rest_threads 0
 * and wide_core 0, then basis_pct in {60, 90, 100}, rest_threads in {128,
 * 256} and wide_core in {2048, 8192} one after the other from the best
 * point) on a prepared batch of
 * the given queries (reps timed executions after one warm-up, results into
 * scratch buffers); the eight fastest are timed again with 3 reps
 * executions, and the fastest of those is kept on the tree and reported.
 * The search obeys tk_set_autotune_limits: candidates abandoned after their
 * warm-up never win, and a spent time budget ends it early. */
tk_status tk_autotune(tk_tree* t, int32_t n, const int64_t* ts, const int64_t* te, int32_t reps,
                      tk_tuning* best, double* best_ms);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of range queries interleaved with appends.
 *
 * After tk_serve_start, queries and appends are submitted from any thread
 * and return a ticket at once; a scheduler thread owned by the tree issues
 * them.  A query sees every append submitted before it (its snapshot T_c),
 * even if that append is still being committed: it is admitted once every
 * node of its hit set has been committed (a query away from the latest
 * appends does not wait for their commits).  Queries are grouped in three size classes by their
 * largest eigenproblem.  Each class runs a stitch launch whose workgroups
 * (at most max_batch: the class's job slots) take admitted queries one at a
 * time from a job ring in host memory that the device maps; a waiting query
 * is admitted, in arrival order, as soon as the ring has a free entry
 * (4 max_batch per class) and the class's workspace (an equal share of
 * ws_budget_bytes, first fit) has room for it, and it runs beside the
 * queries already on the device.  A launch ends after 2 ms without work or
 * 20 ms of age and is relaunched while admitted queries wait.  Appends are
 * committed in groups of up to max_commit_blocks leaf blocks on a stream of
 * their own, concurrently with the queries.  A query's result is
 * bit-identical to tk_query on a tree holding the same slices (same
 * tuning).  While serving, the synchronous calls that read or change the
 * tree return TK_EBUSY.  The engine drives five streams (the tree's, the
 * appends', three classes): run the process with GPU_MAX_HW_QUEUES >= 5
 * (HIP's default is 4), else an append commit that shares a hardware queue
 * with a class's launch waits for it (at 2000 queries/s and 1000 appends/s
 * on the serving workload: query p99 55 ms and append p50 77 ms with 4
 * queues, 26 ms and 31 ms with 8).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t max_batch;          /* job slots (concurrent queries) per class; 0: 256 */
  int32_t max_commit_blocks;  /* leaf blocks per append commit; 0: 64         */
  int64_t ws_budget_bytes;    /* query workspace on the device; 0: 1 GiB      */
  int64_t max_queue;          /* unfinished requests before TK_EBUSY; 0: 2^20 */
} tk_serve_config;

typedef struct {
  int64_t queries, appends;   /* accepted submissions                          */
  int64_t completed;          /* finished requests                             */
  int64_t rejected;           /* refused (queue full or over the budget)       */
  int64_t batches, commits;   /* query launches and append commits issued      */
  int64_t max_batch_seen;     /* most admitted, unfinished queries of a class  */
  int64_t outstanding;        /* submitted, not finished                       */
  int64_t T_submitted;        /* slices submitted                              */
  int64_t T_committed;        /* slices in committed blocks                    */
} tk_serve_stats;

tk_status tk_serve_start(tk_tree* t, const tk_serve_config* cfg);  /* cfg may be NULL */
/* Finish every submitted request, stop the scheduler; synchronous calls work
 * again afterwards (tickets are forgotten). */
tk_status tk_serve_stop(tk_tree* t);
/* res: caller-owned, valid until the ticket is done.  TK_ERANGE if
 * [ts, te) is not inside the snapshot; TK_ENOMEM if the query alone exceeds
 * its class's workspace budget; TK_EBUSY if max_queue requests are open. */
tk_status tk_submit_query(tk_tree* t, int64_t ts, int64_t te, tk_result* res, uint64_t* ticket);
/* A host slice is copied before return; a device slice must stay valid
 * until its ticket is done. */
tk_status tk_submit_append(tk_tree* t, const float* slice, int on_device, uint64_t* ticket);
tk_status tk_poll(tk_tree* t, uint64_t ticket, int32_t* done);  /* TK_EDEVICE if it failed */
tk_status tk_wait(tk_tree* t, uint64_t ticket);
/* Wait until every submitted request is done (without a server: the
 * tree's stream). */
tk_status tk_sync(tk_tree* t);
/* Host times of a request in microseconds since tk_serve_start: submitted,
 * launched (staged, for an append) and done (-1 while pending). */
tk_status tk_ticket_times(tk_tree* t, uint64_t ticket, double* submit_us, double* launch_us,
                          double* done_us);
tk_status tk_serve_stats_get(tk_tree* t, tk_serve_stats* out);

/* Host-only planning helpers (no tree, no device): the pruned hit set of
 * [t_s, t_e) in a tree of committed horizon T built with cfg's leaf_len and
 * theta, and the effective ranks of a range of the given length. */
tk_status tk_hitset_plan(const tk_config* cfg, int64_t T, int64_t ts, int64_t te, tk_hit* out,
                         int32_t cap, int32_t* n);
tk_status tk_effective_ranks(const tk_config* cfg, int64_t length, int32_t* ranks_eff);

/* Library version, "major.minor.patch". */
const char* tk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TUCKET_H */
