// Tucker-ALS from scratch on one long raw range with many workgroups
// (tk_raw_tucker_stream): the iteration of the one-workgroup raw-range
// kernel (Sec. 2's Tucker-ALS: HOSVD of the non-temporal modes, sweeps from
// the temporal mode, the fit stop rule of the stitch), with every pass over
// the range split into spans of consecutive slices, one workgroup each.
//
// Per sweep, with R_n the product of the output ranks other than r_n:
//   * temporal pass: each span's rows of Y = X x_{m>=2} U^(m)T and their
//     R_1 x R_1 Gram; the summed Gram's leading eigenvectors V and values
//     s^2 give U^(1) = Y V diag(1/s) (span by span), made orthonormal by one
//     Cholesky QR step (the r_1 x r_1 Gram of its rows, summed over spans);
//   * mode n >= 2: each span's share X_span x_1 U^(1)[span]^T x_{m != n}
//     U^(m)T of the mode-n product (it is linear in the slices), summed over
//     spans, then the leading left singular vectors of its mode-n unfolding;
//     after the last mode the core and its norm.
// Every reduction over spans runs in a fixed order, so results do not
// depend on timing.  Each pass reads the range once: p reads per sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tk_host.hpp"

namespace tk {

namespace {

constexpr int64_t kStreamSpans = 512;                    // workgroups of a pass, at most
constexpr int64_t kStreamPartBytes = int64_t(1) << 30;   // the partial results of one pass, at most

int64_t align_up(int64_t x) { return (x + 255) & ~int64_t(255); }

}  // namespace

}  // namespace tk

extern "C" tk_status tk_raw_tucker_stream(tk_tree* t, const float* X, int64_t L, tk_result* res) {
  using namespace tk;
  if (!t || !X || !res) return TK_EINVAL;
  if (t->server) return fail(t, TK_EBUSY, "the tree is serving; stop the server first");
  if (t->poisoned) return TK_EDEVICE;
  if (L < 1 || L > (int64_t(1) << 31) - 1) return fail(t, TK_EINVAL, "raw range: bad length");
  if (!res->core) return fail(t, TK_EINVAL, "null core buffer");
  const int p = t->p;
  for (int m = 0; m < p; ++m)
    if (!res->factor[m]) return fail(t, TK_EINVAL, "null factor buffer");
  int32_t rq[MAXP] = {};
  query_ranks(t, L, rq);
  int32_t D[MAXP] = {};
  for (int m = 1; m < p; ++m) D[m] = int32_t(t->view.D[m]);
  int64_t R[MAXP];
  for (int n = 0; n < p; ++n) {
    R[n] = 1;
    for (int m = 0; m < p; ++m)
      if (m != n) R[n] *= rq[m];
  }
  if (R[0] > EIG_MAXK_HOST) return fail(t, TK_EINVAL, "streaming Tucker-ALS: non-temporal ranks multiply above 1024");
  for (int n = 1; n < p; ++n)
    if (D[n] > EIG_MAXK_HOST) return fail(t, TK_EINVAL, "streaming Tucker-ALS: a slice dimension above 1024");
  // partial result of a span, the largest over the passes
  int64_t E = std::max<int64_t>(R[0] * R[0], int64_t(rq[0]) * rq[0]);
  for (int n = 1; n < p; ++n) E = std::max({E, int64_t(D[n]) * D[n], int64_t(D[n]) * R[n]});
  int64_t n_spans = std::min<int64_t>(L, kStreamSpans);
  n_spans = std::min<int64_t>(n_spans, std::max<int64_t>(1, kStreamPartBytes / (E * 8)));
  const int64_t span = (L + n_spans - 1) / n_spans;
  n_spans = (L + span - 1) / span;
  int32_t Dm[MAXP];
  Dm[0] = int32_t(span);
  for (int m = 1; m < p; ++m) Dm[m] = D[m];
  const int64_t t2_off = align_up(projection_max_elems(p, Dm, rq) * 4);
  const int64_t ws_per = 2 * t2_off;
  // one-workgroup steps: eigenproblems up to nmax, other-side vectors
  int64_t nmax = R[0], vmax = 0, zmax = 0, gmax = std::max<int64_t>(R[0] * R[0], int64_t(rq[0]) * rq[0]);
  for (int n = 1; n < p; ++n) {
    nmax = std::max<int64_t>({nmax, D[n], std::min<int64_t>(D[n], R[n])});
    if (D[n] > R[n]) vmax = std::max<int64_t>(vmax, R[n] * rq[n]);
    zmax = std::max<int64_t>(zmax, int64_t(D[n]) * R[n]);
    gmax = std::max<int64_t>(gmax, int64_t(D[n]) * D[n]);
  }
  int cap = 128;
  while (cap > 8 && int64_t(eig_doubles(cap)) * 8 > t->lds_limit - int64_t(leaf_static_lds())) cap -= 8;
  const int n_lds = int(std::min<int64_t>(nmax, cap));
  const size_t lds_bytes = size_t(eig_doubles(n_lds)) * 8;
  const int64_t tmp_off = 0;
  const int64_t eig_off = align_up(eig_tmp_doubles(nmax) * 8);
  const int64_t solve_bytes = eig_off + align_up(eig_doubles(nmax) * 8);
  // small buffers, in doubles: U64 per non-temporal mode, V (R_1 x r_1), s,
  // R^{-1}, the summed Gram, per-span norms, norm and core norm
  int64_t off_u[MAXP] = {};
  int64_t small = 0;
  for (int n = 1; n < p; ++n) {
    off_u[n] = small;
    small += align_up(int64_t(D[n]) * rq[n] * 8) / 8;
  }
  const int64_t off_v = small;
  small += align_up(R[0] * rq[0] * 8) / 8;
  const int64_t off_sv = small;
  small += 64;
  const int64_t off_rinv = small;
  small += align_up(int64_t(rq[0]) * rq[0] * 8) / 8;
  const int64_t off_gram = small;
  small += align_up(gmax * 8) / 8;
  const int64_t off_nx2p = small;
  small += align_up(n_spans * 8) / 8;
  const int64_t off_out = small;
  small += 32;
  const int64_t off_vbuf = small;
  small += align_up(std::max<int64_t>(vmax, 1) * 8) / 8;

  Lane* lane = &t->main;
  tk_status st = TK_OK;
  if ((st = ensure(t, &lane->sx[0], n_spans * ws_per + 256, "streaming projections")) ||
      (st = ensure(t, &lane->sx[1], n_spans * E * 8 + 256, "streaming partial results")) ||
      (st = ensure(t, &lane->sx[2], L * R[0] * 4 + 256, "streaming temporal projection")) ||
      (st = ensure(t, &lane->sx[3], L * rq[0] * 8 + 256, "streaming temporal factor")) ||
      (st = ensure(t, &lane->sx[4], small * 8 + std::max<int64_t>(zmax, 1) * 4 + 512, "streaming small buffers")) ||
      (st = ensure(t, &lane->sx[5], solve_bytes + 256, "streaming solver workspace")))
    return st;
  double* sm = reinterpret_cast<double*>(lane->sx[4].p);
  float* Zr = reinterpret_cast<float*>(sm + small);
  double* part = reinterpret_cast<double*>(lane->sx[1].p);
  double* U1 = reinterpret_cast<double*>(lane->sx[3].p);
  hipStream_t s = lane->stream;

  StreamArgs a{};
  a.X = X;
  a.L = L;
  a.slice = t->slice_elems;
  a.span = span;
  a.p = p;
  for (int m = 0; m < p; ++m) {
    a.D[m] = D[m];
    a.rq[m] = rq[m];
    a.Uf[m] = res->factor[m];
  }
  a.ws = lane->sx[0].p;
  a.ws_per = ws_per;
  a.t2_off = t2_off;
  a.Y = reinterpret_cast<float*>(lane->sx[2].p);
  a.part = part;

  SolveArgs b{};
  b.p = p;
  b.ws = lane->sx[5].p;
  b.tmp_off = tmp_off;
  b.eig_off = eig_off;
  b.n_lds = n_lds;
  b.sv = sm + off_sv;
  b.out = sm + off_out;
  b.vbuf = sm + off_vbuf;
  b.L = L;

  // HOSVD of the non-temporal modes (the first pass also sums ||X||^2)
  for (int n = 1; n < p; ++n) {
    a.skip = n;
    a.part_elems = int64_t(D[n]) * D[n];
    a.nx2 = n == 1 ? sm + off_nx2p : nullptr;
    TK_HIP(t, launch_stream_gram(a, n_spans, s));
    TK_HIP(t, launch_stream_reduce(part, n_spans, a.part_elems, sm + off_gram, nullptr, s));
    b.op = 0;
    b.dims[0] = D[n];
    b.r = rq[n];
    b.gram = sm + off_gram;
    b.U64 = sm + off_u[n];
    b.U32 = res->factor[n];
    TK_HIP(t, launch_stream_solve(b, lds_bytes, s));
  }
  a.nx2 = nullptr;
  TK_HIP(t, launch_stream_reduce(sm + off_nx2p, n_spans, 1, sm + off_out + 1, nullptr, s));

  double host[2] = {0.0, 0.0};
  double fit = 0.0, fit_prev = 0.0, nx2 = 0.0, g2 = 0.0;
  int sweeps = 0, conv = 0;
  for (int it = 1; it <= t->q_max_iter; ++it) {
    // temporal mode
    a.skip = 0;
    a.part_elems = R[0] * R[0];
    TK_HIP(t, launch_stream_project(a, n_spans, s));
    TK_HIP(t, launch_stream_reduce(part, n_spans, a.part_elems, sm + off_gram, nullptr, s));
    b.op = 0;
    b.dims[0] = int32_t(R[0]);
    b.r = rq[0];
    b.gram = sm + off_gram;
    b.U64 = sm + off_v;
    b.U32 = nullptr;
    TK_HIP(t, launch_stream_solve(b, lds_bytes, s));
    a.part_elems = int64_t(rq[0]) * rq[0];
    TK_HIP(t, launch_stream_u1(a, n_spans, sm + off_v, sm + off_sv, U1, s));
    TK_HIP(t, launch_stream_reduce(part, n_spans, a.part_elems, sm + off_gram, nullptr, s));
    b.op = 2;
    b.U64 = sm + off_rinv;
    TK_HIP(t, launch_stream_solve(b, lds_bytes, s));
    TK_HIP(t, launch_stream_u1_fix(a, n_spans, sm + off_rinv, U1, res->factor[0], s));
    // non-temporal modes
    for (int n = 1; n < p; ++n) {
      a.skip = n;
      a.part_elems = int64_t(D[n]) * R[n];
      TK_HIP(t, launch_stream_project(a, n_spans, s));
      TK_HIP(t, launch_stream_reduce(part, n_spans, a.part_elems, nullptr, Zr, s));
      b.op = 1;
      for (int m = 0; m < p; ++m) b.dims[m] = m == n ? D[n] : rq[m];
      b.mode = n;
      b.r = rq[n];
      b.Z = Zr;
      b.U64 = sm + off_u[n];
      b.U32 = res->factor[n];
      b.core = n == p - 1 ? res->core : nullptr;
      TK_HIP(t, launch_stream_solve(b, lds_bytes, s));
    }
    b.core = nullptr;
    TK_HIP(t, hipMemcpyAsync(host, sm + off_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    TK_HIP(t, hipStreamSynchronize(s));
    g2 = host[0];
    nx2 = host[1];
    fit = nx2 > 0.0 ? 1.0 - std::sqrt(std::max(0.0, nx2 - g2)) / std::sqrt(nx2) : 1.0;
    sweeps = it;
    if (it >= 2 && std::fabs(fit - fit_prev) < t->q_tol) {
      conv = 1;
      break;
    }
    fit_prev = fit;
  }
  for (int m = 0; m < TK_MAX_MODES; ++m) res->ranks_eff[m] = m < p ? rq[m] : 0;
  res->fit = fit;
  res->err_model = nx2 > 0.0 ? std::sqrt(std::max(0.0, nx2 - g2)) / std::sqrt(nx2) : 0.0;
  res->norm_ytilde = std::sqrt(nx2);
  res->sweeps = sweeps;
  res->converged = conv;
  res->n_hits = 0;
  return TK_OK;
}
