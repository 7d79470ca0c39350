// Kernel arguments and launchers shared by the kernels and the C API.
#pragma once

#include "tk_common.hpp"

namespace tk {

constexpr int NT_STITCH = 64;  // one wavefront per stitch job
constexpr int NT_LEAF = 256;   // four wavefronts per leaf job

// A job ring that the host feeds while a stitch launch runs (serving): the
// header, the job descriptors, the hits, the statistics and the completion
// words all live in host memory that the device maps (pinned, coherent).
// The host writes job q into slot q mod R and then publishes it by raising
// tail to q + 1; a workgroup claims the next unclaimed job by advancing a
// counter in device memory, runs it, and writes done[slot] = q + 1 when its
// outputs and statistics are visible to the host.  A workgroup stops
// claiming when the host sets stop, when no job has been published for
// idle_ticks of the device's 100 MHz clock, or once the launch is older
// than life_ticks, so every launch ends by itself and the host relaunches
// when jobs are waiting.
struct RingHdr {
  int64_t tail;  // jobs published (host)
  int32_t stop;  // host: claim nothing more
  int32_t slots; // R
};

struct StitchRing {
  RingHdr* hdr;            // device address of the host header
  const Job* jobs;         // R job descriptors (host memory)
  int64_t* done;           // R completion words (host memory)
  int64_t* head;           // jobs claimed (device memory)
  uint64_t idle_ticks;
  uint64_t life_ticks;
};

struct StitchArgs {
  const StoreView* st;
  int p;               // modes of the tree (selects the kernel instantiation)
  const Job* jobs;
  Hit* hits;           // merge jobs: read; query jobs: written by the kernel's own Recall
  char* ws;
  int n_jobs;
  int* queue;          // non-null: persistent launch, workgroups take jobs from this counter
  int n_lds;           // eigenproblems up to n_lds x n_lds run in LDS
  int lds_doubles;     // dynamic LDS of the launch, in doubles; larger eigenproblems keep
                       // their vectors there (eig_vec_doubles(n) <= lds_doubles required)
  int basis_pct;       // span-basis rule (tk_tuning.basis_pct) of the plan
  int max_iter;        // query jobs
  double tol;
  int merge_max_iter;  // merge jobs (node construction)
  double merge_tol;
  int bf16;            // query jobs: BF16 operands in the ALS contractions
  int merge_bf16;      // merge jobs: the same
  int64_t theta_num, theta_den;
  StitchRing ring;     // ring.hdr non-null: jobs come from the host's ring (jobs/n_jobs/queue unused)
};

struct LeafArgs {
  const StoreView* st;
  const LeafJob* jobs;
  char* ws;
  int n_lds;
  int max_iter;
  double tol;
};

struct RawArgs {
  const RawJob* jobs;
  char* ws;
  int p;
  int32_t D[MAXP];  // D[1..p-1]: slice dimensions
  int n_lds;
  int max_iter;
  double tol;
};

// Tucker-ALS on one long raw range with many workgroups (streaming): every
// pass splits the range into spans of `span` consecutive slices, one
// workgroup each, and each workgroup writes its own partial result (slot
// blockIdx.x of `part`, part_elems doubles), summed afterwards in a fixed
// order.
struct StreamArgs {
  const float* X;      // L slices, C order
  int64_t L;
  int64_t slice;       // elements per slice
  int64_t span;        // slices per workgroup (the last takes the rest)
  int p;
  int32_t D[MAXP];     // D[1..p-1]
  int32_t rq[MAXP];    // output ranks
  int skip;            // mode of the pass (0: temporal)
  float* Uf[MAXP];     // FP32 factors; Uf[0] is L x r_1, indexed by slice
  char* ws;            // per-workgroup projection buffers: T1 at 0, T2 at t2_off
  int64_t ws_per, t2_off;
  float* Y;            // temporal pass: the L x R_1 projected rows
  double* part;
  int64_t part_elems;
  double* nx2;         // Gram pass of mode 1: ||X||^2 of each span (or null)
};

// One-workgroup steps between the passes.  op 0: the leading r
// eigenvectors of the n x n FP64 matrix `gram` into U64 (n x r) and U32,
// sqrt of the eigenvalues into sv.  op 1: the leading r left singular
// vectors of mode `mode` of the FP32 tensor Z (dims) into U64 and U32; with
// core set, also core = Z x_mode U^T (mode the last) and out[0] = ||core||^2.
// op 2: R^{-1} (r x r, upper) of the Cholesky factor R of the r x r Gram
// `gram` of U^(1), into U64.
struct SolveArgs {
  int op;
  int p, mode, r;
  int32_t dims[MAXP];
  int64_t L;
  const double* gram;
  const float* Z;
  double* U64;
  float* U32;
  double* sv;
  float* core;
  double* out;
  double* vbuf;      // op 1: other-side vectors
  char* ws;          // eigensolver scratch (TMP at tmp_off, matrix at eig_off)
  int64_t tmp_off, eig_off;
  int n_lds;
};

// threads: 64 (one wavefront per job), 128 or 256 (jobs with large
// eigenproblems).  grid <= n_jobs; with a.queue set the grid may be smaller
// than n_jobs and the queue counter must read 0 at launch (reset_queue).
hipError_t launch_stitch(const StitchArgs& a, int grid, size_t lds_bytes, int threads, hipStream_t stream);
hipError_t launch_reset_queue(int* queue, int n, hipStream_t stream);
// the trim pass over n chunks (trim_gram_kernel)
hipError_t launch_trim(const TrimChunk* chunks, int64_t n, hipStream_t stream);

// Entry points of the stitch kernel's instantiations (block size x mode
// count: 64/128/256 threads, trees of at most 4 or at most MAXP modes), one
// translation unit each (tk_stitch_inst.hip).  launch_stitch dispatches to
// them; occupancy returns 0 when the runtime cannot tell.
#define TK_STITCH_ENTRIES(NTT, PM)                                                                    \
  hipError_t stitch_launch_##NTT##_##PM(const StitchArgs& a, int grid, size_t lds_bytes, hipStream_t stream); \
  hipError_t stitch_set_lds_##NTT##_##PM(size_t bytes);                                              \
  int stitch_occupancy_##NTT##_##PM(size_t lds_bytes);
TK_STITCH_ENTRIES(64, 4)
TK_STITCH_ENTRIES(128, 4)
TK_STITCH_ENTRIES(256, 4)
TK_STITCH_ENTRIES(64, 7)
TK_STITCH_ENTRIES(128, 7)
TK_STITCH_ENTRIES(256, 7)
#undef TK_STITCH_ENTRIES

hipError_t launch_leaf(const LeafArgs& a, int n_jobs, size_t lds_bytes, hipStream_t stream);
// one NT_LEAF workgroup per raw range
hipError_t launch_raw(const RawArgs& a, int n_jobs, size_t lds_bytes, hipStream_t stream);
hipError_t set_lds_limits(size_t stitch_bytes, size_t leaf_bytes);
// streaming Tucker-ALS passes: one NT_LEAF workgroup per span
hipError_t launch_stream_gram(const StreamArgs& a, int64_t n_spans, hipStream_t stream);
hipError_t launch_stream_project(const StreamArgs& a, int64_t n_spans, hipStream_t stream);
// U64 rows [span b] = Y rows V diag(1 / sv) (V: R_1 x r), the rows' partial
// Gram into part
hipError_t launch_stream_u1(const StreamArgs& a, int64_t n_spans, const double* V, const double* sv, double* U64,
                            hipStream_t stream);
// U64 rows <- U64 rows Rinv (Rinv r_1 x r_1 upper triangular), and U32 = U64
hipError_t launch_stream_u1_fix(const StreamArgs& a, int64_t n_spans, const double* Rinv, double* U64, float* U32,
                                hipStream_t stream);
// out = sum over n_parts of part[b][e] (FP64, in b order), into out64 and/or out32
hipError_t launch_stream_reduce(const double* part, int64_t n_parts, int64_t E, double* out64, float* out32,
                                hipStream_t stream);
hipError_t launch_stream_solve(const SolveArgs& a, size_t lds_bytes, hipStream_t stream);
// workgroups of the stitch kernel with `threads` threads and lds_bytes of
// dynamic LDS that one CU holds at once
int stitch_blocks_per_cu(int threads, size_t lds_bytes);
size_t stitch_static_lds();
size_t leaf_static_lds();

}  // namespace tk
