// Kernel arguments and launchers shared by the kernels and the C API.
#pragma once

#include "tk_common.hpp"

namespace tk {

constexpr int NT_STITCH = 64;        // one wavefront per stitch job
constexpr int NT_STITCH_WIDE = 256;  // four wavefronts for jobs with large eigenproblems
constexpr int NT_LEAF = 256;    // four wavefronts per leaf job

struct StitchArgs {
  const StoreView* st;
  const Job* jobs;
  const Hit* hits;
  char* ws;
  int n_lds;           // eigenproblems up to n_lds x n_lds run in LDS
  int max_iter;        // query jobs
  double tol;
  int merge_max_iter;  // merge jobs (node construction)
  double merge_tol;
};

struct LeafArgs {
  const StoreView* st;
  const LeafJob* jobs;
  char* ws;
  int n_lds;
  int max_iter;
  double tol;
};

hipError_t launch_stitch(const StitchArgs& a, int n_jobs, size_t lds_bytes, bool wide, hipStream_t stream);
hipError_t launch_leaf(const LeafArgs& a, int n_jobs, size_t lds_bytes, hipStream_t stream);
hipError_t set_lds_limits(size_t stitch_bytes, size_t leaf_bytes);
size_t stitch_static_lds();
size_t leaf_static_lds();

}  // namespace tk
