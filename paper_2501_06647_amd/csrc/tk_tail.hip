// Provisional leaf of the incomplete block: queries reaching past the last
// complete block (1 <= m < leaf_len slices in the staging buffer) stitch it
// as a partial hit of the next leaf slot.  The block's Tucker-ALS runs with
// the raw-range kernel at the node ranks clipped to m; this file places the
// compact result into the slot zero-padded to the slot's shapes (extra core
// entries, factor columns and temporal rows are zero, so the represented
// tensor is the same and a trim of its m rows drops the padding).  The slot
// is rewritten by the real leaf when the block completes.
#include <hip/hip_runtime.h>

#include "tk_host.hpp"

namespace tk {

namespace {

struct TailPlace {
  const StoreView* st;
  int64_t b;   // leaf slot
  int32_t m;   // slices of the incomplete block
  int32_t p;
  int32_t rq[MAXP];          // ranks of the compact decomposition
  const float* core;         // prod(rq), C order
  const float* fac[MAXP];    // fac[0]: m x rq[0]; fac[n]: D_n x rq[n]
};

__global__ void place_tail_kernel(TailPlace a) {
  const StoreView& st = *a.st;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  const int p = a.p;
  const int32_t* rk = st.rk[0];
  const int64_t ce = st.core_elems[0];
  float* core = st.core[0] + a.b * ce;
  for (int64_t e = tid; e < ce; e += nth) {
    int64_t rem = e;
    int64_t idx[MAXP];
    for (int n = p - 1; n >= 0; --n) {
      idx[n] = rem % rk[n];
      rem /= rk[n];
    }
    bool in = true;
    int64_t src = 0;
    for (int n = 0; n < p; ++n) {
      in = in && idx[n] < a.rq[n];
      src = src * a.rq[n] + idx[n];
    }
    core[e] = in ? a.core[src] : 0.0f;
  }
  for (int n = 1; n < p; ++n) {
    const int64_t R = rk[n];
    float* dst = st.fac[0][n] + a.b * st.D[n] * R;
    for (int64_t e = tid; e < st.D[n] * R; e += nth) {
      const int64_t d = e / R, j = e % R;
      dst[e] = j < a.rq[n] ? a.fac[n][d * a.rq[n] + j] : 0.0f;
    }
  }
  const int64_t R0 = rk[0];
  float* plane = st.plane[0] + a.b * st.ell * R0;
  for (int64_t e = tid; e < st.ell * R0; e += nth) {
    const int64_t i = e / R0, j = e % R0;
    plane[e] = (i < a.m && j < a.rq[0]) ? a.fac[0][i * a.rq[0] + j] : 0.0f;
  }
}

}  // namespace

tk_status provisional_leaf(tk_tree* t) {
  const int64_t m = t->T - t->Tb * t->ell;
  if (m <= 0) return fail(t, TK_ERANGE, "no incomplete block");
  if (t->prov_T == t->T) return TK_OK;
  const int p = t->p;
  RawJob jb{};
  jb.X = t->block_buf;
  jb.L = m;
  effective_ranks(p, m, t->view.D, t->cfg.ranks, jb.rq);
  int32_t Dm[MAXP];
  Dm[0] = int32_t(m);
  for (int n = 1; n < p; ++n) Dm[n] = int32_t(t->view.D[n]);
  int cap = 128;
  while (cap > 8 && int64_t(eig_doubles(cap)) * 8 > t->lds_limit - int64_t(leaf_static_lds())) cap -= 8;
  LeafLayout lo;
  raw_layout(p, Dm, jb.rq, 1 << 30, &lo);
  const int n_lds = lo.neig < cap ? lo.neig : cap;
  raw_layout(p, Dm, jb.rq, n_lds, &lo);
  int64_t out_elems = 1;
  for (int n = 0; n < p; ++n) out_elems *= jb.rq[n];
  int64_t off[MAXP + 1];
  off[0] = out_elems;
  for (int n = 0; n < p; ++n) off[n + 1] = off[n] + int64_t(Dm[n]) * jb.rq[n];
  Lane* lane = &t->main;
  tk_status st = ensure(t, &t->prov_out, off[p] * 4 + 256, "provisional leaf");
  if (st) return st;
  st = ensure(t, &lane->leaf_ws, lo.total + 256, "workspace");
  if (st) return st;
  st = ensure(t, &lane->leaf_jobs, int64_t(sizeof(RawJob)), "jobs");
  if (st) return st;
  float* out = reinterpret_cast<float*>(t->prov_out.p);
  jb.out_core = out;
  for (int n = 0; n < p; ++n) jb.out_fac[n] = out + off[n];
  jb.stats = nullptr;
  jb.ws_off = 0;
  TK_HIP(t, hipMemcpyAsync(lane->leaf_jobs.p, &jb, sizeof(RawJob), hipMemcpyHostToDevice, t->stream));
  RawArgs a{};
  a.jobs = reinterpret_cast<const RawJob*>(lane->leaf_jobs.p);
  a.ws = lane->leaf_ws.p;
  a.p = p;
  for (int n = 1; n < p; ++n) a.D[n] = int32_t(t->view.D[n]);
  a.n_lds = n_lds;
  a.max_iter = t->cfg.max_iter;
  a.tol = t->cfg.tol;
  TK_HIP(t, launch_raw(a, 1, size_t(eig_doubles(n_lds)) * 8, t->stream));
  TailPlace pl{};
  pl.st = t->dview;
  pl.b = t->Tb;
  pl.m = int32_t(m);
  pl.p = p;
  for (int n = 0; n < p; ++n) {
    pl.rq[n] = jb.rq[n];
    pl.fac[n] = jb.out_fac[n];
  }
  pl.core = out;
  hipLaunchKernelGGL(place_tail_kernel, dim3(64), dim3(256), 0, t->stream, pl);
  TK_HIP(t, hipGetLastError());
  // the job descriptor upload above is from a stack copy: finish before it goes
  TK_HIP(t, hipStreamSynchronize(t->stream));
  t->prov_T = t->T;
  return TK_OK;
}

}  // namespace tk
