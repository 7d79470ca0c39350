// The stitch kernel (gfx950): one job (a range query or the merge of two
// children) per workgroup.  Each (block size, mode count) instantiation is
// compiled in a translation unit of its own (tk_stitch_inst.hip), so the
// build runs them in parallel.
//
// A job is a range query (Sec. 6.1: Recall's hits -> partial-hit trims,
// Eq. "partial-tucker" -> Alg. "stitch") or the merge of two children when a
// node completes (Alg. "insert").
//
// Alg. "stitch" is Tucker-ALS on the concatenation Y~ of the hit pieces,
// Y~_i = H~_i x_1 V~_i^(1) ... x_p V~_i^(p).  The kernel runs it in exact
// reduced coordinates:
//   * temporal mode: the blocks V~_i^(1) are orthonormal, so the leading left
//     singular vectors of Z^(1) (Eq. "stitch-temp-2") are
//     blockdiag(V~_i^(1)) P with P those of the small stacked matrix
//     M = [mat_1(H~_i x_{m>=2} (U^(m)T V~_i^(m)))]_i, and
//     U^(1)_{[t_{i-1},t_i)}^T V~_i^(1) = P_i^T;
//   * mode n >= 2: Z^(n) (Eq. "stitch-nontemp-3") lies in the span of
//     [V~_1^(n) .. V~_s^(n)]; with B an orthonormal basis of that span and
//     C_i = B^T V~_i^(n), B^T Z^(n) = sum_i C_i mat_n(W_i^(n)) and
//     U^(n) = B P_n, U^(n)T V~_i^(n) = P_n^T C_i.
// The leading singular vectors come from the Gram of the small matrix and an
// FP64 symmetric eigensolver (Householder tridiagonalisation, bisection,
// inverse iteration).  Partial hits are trimmed through a pivoted Cholesky
// factor of the Gram of the sliced rows (an exact orthonormal factorisation,
// equal to the QR of Eq. "partial-tucker" up to a permutation of the piece's
// core rows), and the span bases come from a pivoted Cholesky factor of the
// factors' Gram.  Full-size factors are formed once, in FP64, when the
// result is written.
#pragma once

#include "tk_device.hpp"
#include "tk_internal.hpp"

namespace tk {

__device__ __forceinline__ void wg_copy(float* dst, const float* src, int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

__device__ __forceinline__ int64_t prod_range(const int32_t* d, int lo, int hi) {
  int64_t r = 1;
  for (int m = lo; m < hi; ++m) r *= d[m];
  return r;
}

// Phase timer: thread 0 accumulates the 100 MHz wall clock between marks
// (state in LDS, so it costs no registers over the kernel's lifetime).
struct PhaseClock {
  uint64_t last;
  uint64_t acc[STAT_NPHASE];
  __device__ __forceinline__ void start() {
    if (threadIdx.x == 0) {
      last = wall_clock64();
      for (int i = 0; i < STAT_NPHASE; ++i) acc[i] = 0;
    }
  }
  __device__ __forceinline__ void mark(int ph) {
    if (threadIdx.x == 0) {
      const uint64_t now = wall_clock64();
      acc[ph] += now - last;
      last = now;
    }
  }
  __device__ __forceinline__ void store(double* stats) const {
    if (threadIdx.x == 0 && stats)
      for (int i = 0; i < STAT_NPHASE; ++i) stats[STAT_PHASE + i] = double(acc[i]) * 0.01;
  }
};

// PM: the most modes the instantiation handles (its per-mode arrays)
template <int PM>
struct StitchShared {
  PhaseClock clk;
  EigCounters ec;
  int64_t recall_stack[RECALL_STACK];
  int32_t kp[MAXHITS];              // temporal rank of each piece after its trim
  int32_t koff[MAXHITS + 1];        // offsets of the pieces in the stacked temporal coordinates
  int32_t roff[PM][MAXHITS + 1];    // offsets of the pieces' columns in C^(n)
  int32_t q[PM];                    // size of the reduced coordinates of mode n
  int32_t basis[PM];                // 1: C^(n) from the Cholesky basis; 0: C^(n) = V~
  int32_t warm[PM];                 // 1: mode n's next eigensolve starts from the vectors in P_n;
                                    // 2, 3: it runs in full, later sweeps' may start warm again
                                    // (2: no start written, 3: a start failed); 0: all in full
  double red[8];
  int redi[4];
};

// Stitch instantiations: up to four modes (the per-mode arrays and the
// register budget of the three- and four-way workloads), and up to MAXP
// modes.  The many-mode one runs small TTM products (at most 8 outputs from
// at most 8 inputs per fiber, as in rank-5 chains over 5 to 7 modes) one
// fiber per lane: a 16 x 16 matrix-core tile would be mostly padding.
constexpr int PM_FEW = 4;

template <int PM>
__device__ __forceinline__ void stitch_one(const StoreView& st, const Job& job, const Hit* hits, char* ws, int n_lds,
                           int lds_doubles, int basis_pct, int max_iter, double tol, bool lowp, StitchShared<PM>& sh,
                           double* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int p = st.p;
  const int s = job.s;
  const int32_t* rq = job.rq;

  // One entire hit at the node's own ranks: the range is a stored node;
  // return it verbatim.
  bool node_ranks = s == 1 && !hits[0].partial;
  for (int n = 0; n < p && node_ranks; ++n) node_ranks = rq[n] == st.rk[hits[0].level][n];
  if (node_ranks) {
    const Hit h = hits[0];
    const int lev = h.level;
    wg_copy(job.out_core, st.core[lev] + h.index * st.core_elems[lev], st.core_elems[lev]);
    for (int n = 1; n < p; ++n)
      wg_copy(job.out_fac[n], st.fac[lev][n] + h.index * fac_elems(st, lev, n), fac_elems(st, lev, n));
    const int64_t row0 = (h.index << lev) * st.ell;
    wg_copy(job.out_fac[0], st.plane[lev] + row0 * st.rk[lev][0], (st.ell << lev) * st.rk[lev][0]);
    if (tid == 0 && job.stats) {
      job.stats[STAT_FIT] = -1.0;
      job.stats[STAT_ERR] = -1.0;
      job.stats[STAT_NORM] = -1.0;
      job.stats[STAT_SWEEPS] = 0.0;
      job.stats[STAT_CONV] = 1.0;
      job.stats[STAT_HITS] = 1.0;
      job.stats[STAT_STATUS] = 0.0;
    }
    return;
  }

  PhaseClock& clk = sh.clk;
  EigCounters& ec = sh.ec;
  if (tid == 0) {
    ec.calls = ec.sweeps = ec.values_ticks = ec.tail_ticks = ec.fallbacks = ec.tri_ticks = ec.invit_ticks = 0;
    ec.warm = ec.warm_fail = ec.warm_steps = ec.warm_ticks = ec.warm_rr_ticks = 0;
  }
  clk.start();
  // the layout record lives at the head of the workspace
  StitchLayout* lop = reinterpret_cast<StitchLayout*>(ws);
  if (tid == 0) stitch_layout(st, hits, s, rq, n_lds, lop, job.pretrim);
  __threadfence_block();
  __syncthreads();
  const StitchLayout& lo = *lop;
  if (lo.total > job.ws_bytes) {
    if (tid == 0 && job.stats) job.stats[STAT_STATUS] = 2.0;
    return;
  }
  const int eneed = stitch_eig_need(lo, st, basis_pct);
  if (eneed > n_lds && eig_vec_doubles(eneed) > lds_doubles) {  // launched with too little LDS
    if (tid == 0 && job.stats) job.stats[STAT_STATUS] = 3.0;
    return;
  }
  double* red = sh.red;
  // the ALS contractions (TTM chains, Z^(n), core update) and their Grams:
  // FP32 on the matrix cores, or BF16 operands with FP32 accumulation.  In
  // the BF16 mode the last mode's chain and the core update keep FP32
  // operands: the sweep's stop test compares fits through |Y~|^2 - |G|^2,
  // which cancels to a few per mille of |Y~|^2 at the workloads' fits, so
  // the BF16 rounding of |G|^2 (~2^-9 relative) would exceed the tolerance
  // and hold the stop back for extra sweeps.
  bool lp = lowp;
  auto ttm = [&](const float* X, int64_t a, int r, int64_t b, const float* A, int64_t as, int64_t bs, int m,
                 float* Y, bool acc) {
    if (lp) mode_product_bf16(X, a, r, b, A, as, bs, m, Y, acc);
    else if (PM > PM_FEW && m <= 8 && r <= 8) mode_product_fiber<float, float, float, float, 8>(X, a, r, b, A, as, bs, m, Y, acc);
    else mode_product(X, a, r, b, A, as, bs, m, Y, acc);
  };
  auto gram = [&](const float* X, int64_t a, int q, int64_t b, double* G, int ld) {
    if (lp) gram_mode_bf16(X, a, q, b, G, ld);
    else gram_mode_mfma(X, a, q, b, G, ld);
  };
  auto Fp = [&](int64_t off) { return reinterpret_cast<float*>(ws + off); };
  auto Dp = [&](int64_t off) { return reinterpret_cast<double*>(ws + off); };
  double* TMP = Dp(lo.TMP);
  // Run f on the eigen/Cholesky buffer (matrix part, vector part): both in
  // LDS when the problem fits, else the matrix in the job's global buffer and
  // the vectors in LDS.  Calling f from two branches lets each inlined copy
  // address its buffers directly (LDS instructions where they are in LDS).
  auto with_buf = [&](int n, auto&& f) {
    if (n <= n_lds) f(lds, lds + int64_t(n) * n);
    else f(Dp(lo.EIG), lds);
  };
  // the same for a mode's eigenproblem, which may exceed the planned size
  // (a rank-deficient basis falls back to D_n): vectors in LDS only when
  // the launch has room for them
  auto with_eig_buf = [&](int n, auto&& f) {
    if (n <= n_lds) f(lds, lds + int64_t(n) * n);
    else if (eig_vec_doubles(n) <= lds_doubles) f(Dp(lo.EIG), lds);
    else f(Dp(lo.EIG), Dp(lo.EIG) + int64_t(n) * n);
  };
  // LDS left free behind an eigen buffer of size n placed by with_buf /
  // with_eig_buf (the eigensolver keeps its LU rows there when they fit)
  auto eig_free = [&](int n, double** p) -> int64_t {
    int64_t used = 0;
    if (n <= n_lds) used = int64_t(n) * n + eig_vec_doubles(n);
    else if (eig_vec_doubles(n) <= lds_doubles) used = eig_vec_doubles(n);
    else used = lds_doubles;
    *p = lds + used;
    return lds_doubles - used;
  };
  // An eigensolve for mode `mode` (Gram n x n in Wm, vector buffer Wv, as
  // with_buf / with_eig_buf placed them): the k leading eigenvectors into
  // P_mode.  The Gram changes little from sweep to sweep, so the previous
  // sweep's vectors (or a start written there) begin a subspace iteration
  // that is kept when its certificate holds (eig_top_warm); otherwise, and
  // for the rest of the job's sweeps once a start has failed, the full
  // solver runs.  A start refused for lack of a gap after the k-th
  // eigenvalue (node ranks above the data's rank: no start converges)
  // rules out the mode's later starts in the job; one refused otherwise
  // (a start too far off) only its starts until the next sweep begins
  // afresh (after the HOSVD initialisation, after the first temporal
  // solve).  The iteration's
  // k x k matrices go to the LDS behind the Gram (the eigensolver's vector
  // part, sized for them up to WARM_SMALL_K), its two n x k blocks behind
  // those when they fit, else to TMP.
  auto sweep_eig = [&](int mode, double* Wm, double* Wv, int n, int k) {
    double* E = Dp(lo.Pd[mode]);
    if (sh.warm[mode] == 1 && n > k && k <= 32) {
      const int64_t used = n <= n_lds ? int64_t(n) * n : 0;
      const int64_t nsm = warm_small_doubles(k), nqy = 2 * int64_t(n) * k;
      if (lds_doubles - used >= nsm) {
        double* sm = lds + used;
        double* qy = lds_doubles - used - nsm >= nqy ? sm + nsm : (nqy <= eig_tmp_doubles(n) ? TMP : nullptr);
        if (qy) {
          const int got = eig_top_warm(Wm, n, k, E, k, qy, sm, red, &ec);
          if (got > 0) return;
          if (tid == 0) sh.warm[mode] = got < 0 ? 0 : 3;
        }
      }
    }
    double* lf = nullptr;
    const int64_t nf = eig_free(n, &lf);
    eig_top(Wm, n, k, E, k, red, TMP, &ec, Wv, lf, nf);
  };

  // ---- trims (Eq. "partial-tucker") and |Y~|^2 ------------------------------
  double ny2 = 0.0;
  int64_t tg_off = 0;  // this hit's chunk Grams in TG (pretrim)
  for (int i = 0; i < s; ++i) {
    const Hit h = hits[i];
    const int lev = h.level;
    const int k = st.rk[lev][0];
    int64_t R = 1;
    for (int n = 1; n < p; ++n) R *= st.rk[lev][n];
    const float* H = st.core[lev] + h.index * st.core_elems[lev];
    if (!h.partial) {
      if (tid == 0) sh.kp[i] = k;
      double part = 0.0;
      for (int64_t e = tid; e < int64_t(k) * R; e += nt) part += double(H[e]) * double(H[e]);
      ny2 += block_sum(part, red);
      continue;
    }
    // rows [a, a+l) of V^(1) = Q~ R~ through a pivoted Cholesky of their Gram
    const float* V = st.plane[lev] + ((h.index << lev) * st.ell + h.a) * k;
    float* Rt = Fp(lo.T1);  // R~, kp x k
    int kp = 0;
    with_buf(k, [&](double* Gm, double*) {
      if (job.pretrim) {  // the trim pass summed the rows' Gram by chunks: add them in order
        const double* P = Dp(lo.TG) + tg_off;
        const int64_t nc = trim_chunks(h.l);
        for (int e = tid; e < k * k; e += nt) {
          double acc = 0.0;
          for (int64_t c = 0; c < nc; ++c) acc += P[c * k * k + e];
          Gm[e] = acc;
        }
        __syncthreads();
        tg_off += nc * k * k;
      } else {
        gram_rows(V, h.l, k, Gm, k, Dp(lo.D1));
      }
      double* col = Gm + k * k;
      int* piv = reinterpret_cast<int*>(Gm + k * k + k);
      kp = pchol_inplace(Gm, k, 1e-12, piv, red, sh.redi);
      pchol_basis_inplace<float>(Gm, piv, k, kp, Rt, k, Dp(lo.F[i]), k, col);
    });
    float* Ht = Fp(lo.Ht[i]);
    mode_product(H, 1, k, R, Rt, k, 1, kp, Ht, false);
    double part = 0.0;
    for (int64_t e = tid; e < int64_t(kp) * R; e += nt) part += double(Ht[e]) * double(Ht[e]);
    ny2 += block_sum(part, red);
    if (tid == 0) sh.kp[i] = kp;
    __syncthreads();
  }
  clk.mark(0);
  if (tid == 0) {
    sh.koff[0] = 0;
    for (int i = 0; i < s; ++i) sh.koff[i + 1] = sh.koff[i] + sh.kp[i];
    for (int n = 1; n < p; ++n) {
      sh.roff[n][0] = 0;
      for (int i = 0; i < s; ++i) sh.roff[n][i + 1] = sh.roff[n][i] + st.rk[hits[i].level][n];
    }
  }
  __syncthreads();
  auto core_of = [&](int i) -> const float* {
    const Hit& h = hits[i];
    return h.partial ? Fp(lo.Ht[i]) : st.core[h.level] + h.index * st.core_elems[h.level];
  };
  auto fac_of = [&](int i, int n) -> const float* {
    const Hit& h = hits[i];
    return st.fac[h.level][n] + h.index * fac_elems(st, h.level, n);
  };
  auto A_off = [&](int i, int n) -> int64_t {  // offset of U^(n)T V~_i^(n) = P_n^T C_i, rq_n x r_i^(n)
    int64_t off = 0;
    for (int m = 1; m < n; ++m) off += int64_t(rq[m]) * st.rk[hits[i].level][m];
    return off;
  };
  auto hit_of_col = [&](int n, int c) {  // the hit whose mode-n factor holds column c of V_cat
    int i = 0;
    while (c >= sh.roff[n][i + 1]) ++i;
    return i;
  };
  auto vcat = [&](int n, int64_t dd, int c) -> float {  // V_cat[dd][c]
    const int i = hit_of_col(n, c);
    return fac_of(i, n)[dd * st.rk[hits[i].level][n] + (c - sh.roff[n][i])];
  };

  // ---- orthonormal bases of the non-temporal spans -----------------------------
  for (int n = 1; n < p; ++n) {
    const int sr = lo.sr[n];
    const int64_t Dn = st.D[n];
    float* C = Fp(lo.C[n]);  // q x sr, leading dimension sr
    double* C64 = Dp(lo.C64[n]);
    int use_basis = 0;
    if (span_basis(sr, Dn, basis_pct)) {
      with_buf(sr, [&](double* Gm, double*) {
        // Gram of V_cat = [V~_1^(n) .. V~_s^(n)] over its D_n rows, FP64 on
        // the matrix cores, exactly symmetric (the upper triangle mirrored)
        auto vcol = [&](int c, const float** ptr, int64_t* stride) {
          const int i = hit_of_col(n, c);
          *stride = st.rk[hits[i].level][n];
          *ptr = fac_of(i, n) + (c - sh.roff[n][i]);
        };
        if (sr <= 16) gram_cols_panel<1>(int(Dn), sr, vcol, Gm, sr);
        else if (sr <= 32) gram_cols_panel<2>(int(Dn), sr, vcol, Gm, sr);
        else if (sr <= 48) gram_cols_panel<3>(int(Dn), sr, vcol, Gm, sr);
        else {
          gemm_f64(sr, sr, int(Dn), [&](int x, int dd) { return vcat(n, dd, x); },
                   [&](int dd, int y) { return vcat(n, dd, y); }, [&](int x, int y, double v) { Gm[x * sr + y] = v; });
          for (int e = tid; e < sr * sr; e += nt) {
            const int x = e / sr, y = e % sr;
            if (y < x) Gm[e] = Gm[y * sr + x];
          }
          __syncthreads();
        }
        double* col = Gm + sr * sr;
        int* piv = reinterpret_cast<int*>(Gm + sr * sr + sr);
        const int q = pchol_inplace(Gm, sr, 1e-11, piv, red, sh.redi);
        if (q >= rq[n]) {
          use_basis = 1;
          pchol_basis_inplace<double>(Gm, piv, sr, q, C64, sr, Dp(lo.Fn[n]), sr, col);
          for (int e = tid; e < q * sr; e += nt) C[e] = float(C64[e]);
          if (tid == 0) sh.q[n] = q;
        }
      });
    }
    if (!use_basis) {
      for (int64_t e = tid; e < Dn * sr; e += nt) {
        const int64_t dd = e / sr;
        const int c = int(e % sr);
        int i = 0;
        while (c >= sh.roff[n][i + 1]) ++i;
        const int r = st.rk[hits[i].level][n];
        C[e] = fac_of(i, n)[dd * r + (c - sh.roff[n][i])];
        C64[e] = double(C[e]);
      }
      if (tid == 0) sh.q[n] = int32_t(Dn);
    }
    if (tid == 0) sh.basis[n] = use_basis;
    __syncthreads();
  }
  clk.mark(1);

  // P_n^T C_i for every piece (mode n >= 1), FP32 copy of P_n
  auto update_A = [&](int n) {
    const int q = sh.q[n], sr = lo.sr[n], r_out = rq[n];
    const double* P = Dp(lo.Pd[n]);
    const double* C64 = Dp(lo.C64[n]);
    // [A_1 .. A_s] = P_n^T C^(n) (r_out x sr); A_i is stored r_out x r_i
    gemm_f64(r_out, sr, q, [&](int c, int dd) { return P[dd * r_out + c]; },
             [&](int dd, int col) { return C64[int64_t(dd) * sr + col]; },
             [&](int c, int col, double v) {
               const int i = hit_of_col(n, col);
               const int r = st.rk[hits[i].level][n];
               Fp(lo.A[i])[A_off(i, n) + int64_t(c) * r + (col - sh.roff[n][i])] = float(v);
             });
    float* Pf = Fp(lo.Pf[n]);
    for (int e = tid; e < q * r_out; e += nt) Pf[e] = float(P[e]);
    __syncthreads();
  };

  // The longest hit carries most of Y~: its own leading vectors start the
  // subspace iterations that have no previous sweep (its mode-n factor's
  // coordinates for the HOSVD initialisation, its rows of the stacked
  // temporal coordinates for the first temporal solve); the certificate of
  // eig_top_warm decides as for any start.
  int dom = 0;
  for (int i = 1; i < s; ++i)
    if (hits[i].l > hits[dom].l) dom = i;

  // ---- HOSVD initialisation of U^(2..p) (Gram of Y~ in reduced coordinates)
  for (int n = 1; n < p; ++n) {
    const int q = sh.q[n], sr = lo.sr[n];
    {
      const int rd = st.rk[hits[dom].level][n], c0 = sh.roff[n][dom];
      const int r = rq[n];
      const double* C64 = Dp(lo.C64[n]);
      double* P = Dp(lo.Pd[n]);
      if (rd >= r)
        for (int e = tid; e < q * r; e += nt) P[e] = C64[int64_t(e / r) * sr + c0 + e % r];
      if (tid == 0) sh.warm[n] = rd >= r ? 1 : 2;
      __syncthreads();
    }
    with_eig_buf(q, [&](double* Wm, double* Wv) {
    for (int e = tid; e < q * q; e += nt) Wm[e] = 0.0;
    __syncthreads();
    double* S = Dp(lo.S);
    double* T = Dp(lo.D1);  // C_i S_i, q x r
    const double* C64 = Dp(lo.C64[n]);
    for (int i = 0; i < s; ++i) {
      const int lev = hits[i].level;
      const int r = st.rk[lev][n];
      int32_t dims[PM];
      dims[0] = sh.kp[i];
      for (int m = 1; m < p; ++m) dims[m] = st.rk[lev][m];
      gram_mode_mfma(core_of(i), prod_range(dims, 0, n), r, prod_range(dims, n + 1, p), S, r);
      const int c0 = sh.roff[n][i];
      // T = C_i S_i (q x r), then Wm += T C_i^T
      gemm_f64(q, r, r, [&](int dd, int c) { return C64[int64_t(dd) * sr + c0 + c]; },
               [&](int c, int j) { return S[c * r + j]; }, [&](int dd, int j, double v) { T[dd * r + j] = v; });
      gemm_f64(q, q, r, [&](int dd, int j) { return T[dd * r + j]; },
               [&](int j, int d2) { return C64[int64_t(d2) * sr + c0 + j]; },
               [&](int dd, int d2, double v) { Wm[dd * q + d2] += v; });
    }
    sweep_eig(n, Wm, Wv, q, rq[n]);
    });
    update_A(n);
  }
  {
    const int r0 = rq[0], k0 = sh.kp[dom], o0 = sh.koff[dom];
    const int sk = sh.koff[s];
    double* P0 = Dp(lo.Pd[0]);
    if (k0 >= r0)
      for (int e = tid; e < sk * r0; e += nt) P0[e] = (e / r0 - o0 == e % r0) ? 1.0 : 0.0;
    if (tid == 0)
      for (int n = 0; n < p; ++n) sh.warm[n] = n > 0 ? int(sh.warm[n] != 0) : (k0 >= r0 ? 1 : 2);
    __syncthreads();
  }
  clk.mark(2);

  // ---- ALS sweeps (Alg. "stitch") ---------------------------------------------
  int64_t Rhat[PM];
  for (int n = 0; n < p; ++n) {
    Rhat[n] = 1;
    for (int m = 0; m < p; ++m)
      if (m != n) Rhat[n] *= rq[m];
  }
  float* T1 = Fp(lo.T1);
  float* T2 = Fp(lo.T2);
  float* G = Fp(lo.G);
  double fit_prev = 0.0, fit = 0.0;
  int sweeps = 0, conv = 0;
  double g2 = 0.0;
  for (int it = 1; it <= max_iter; ++it) {
    lp = lowp;
    // temporal mode: M = [mat_1(H~_i x_{m>=2} A_i^(m))]_i, P_0 = leading eigvecs of M M^T
    float* M = Fp(lo.M);
    for (int i = 0; i < s; ++i) {
      const int lev = hits[i].level;
      int32_t dims[PM];
      dims[0] = sh.kp[i];
      for (int m = 1; m < p; ++m) dims[m] = st.rk[lev][m];
      const float* cur = core_of(i);
      for (int n = 1; n < p; ++n) {
        float* out = (n == p - 1) ? M + int64_t(sh.koff[i]) * Rhat[0] : ((n & 1) ? T1 : T2);
        ttm(cur, prod_range(dims, 0, n), dims[n], prod_range(dims, n + 1, p),
            Fp(lo.A[i]) + A_off(i, n), dims[n], 1, rq[n], out, false);
        dims[n] = rq[n];
        cur = out;
      }
    }
    const int sk = sh.koff[s];
    with_buf(sk, [&](double* Wm, double* Wv) {
      gram(M, 1, sk, Rhat[0], Wm, sk);
      clk.mark(3);
      sweep_eig(0, Wm, Wv, sk, rq[0]);
    });
    if (tid == 0 && it == 1) sh.warm[0] = sh.warm[0] != 0;
    float* P0f = Fp(lo.Pf[0]);
    {
      const double* P0 = Dp(lo.Pd[0]);
      for (int e = tid; e < sk * rq[0]; e += nt) P0f[e] = float(P0[e]);
      __syncthreads();
    }
    clk.mark(4);
    // non-temporal modes: K_n = sum_i W_i^(n) x_n C_i, P_n = leading eigvecs of its Gram
    float* K = Fp(lo.K);
    float* Wst = Fp(lo.WS);
    for (int n = 1; n < p; ++n) {
      lp = lowp && n < p - 1;
      const int q = sh.q[n];
      int32_t kd[PM];
      for (int m = 0; m < p; ++m) kd[m] = rq[m];
      kd[n] = q;
      const int64_t ka = prod_range(kd, 0, n), kb = prod_range(kd, n + 1, p);
      for (int i = 0; i < s; ++i) {
        const int lev = hits[i].level;
        int32_t dims[PM];
        dims[0] = sh.kp[i];
        for (int m = 1; m < p; ++m) dims[m] = st.rk[lev][m];
        const float* cur = core_of(i);
        float* bufs[2] = {T1, T2};
        int nb = 0;
        // x_1 P_i^T : A(c, j) = P0[(koff_i + j) rq_0 + c]
        ttm(cur, 1, dims[0], prod_range(dims, 1, p), P0f + int64_t(sh.koff[i]) * rq[0], 1, rq[0],
                     rq[0], bufs[nb], false);
        dims[0] = rq[0];
        cur = bufs[nb];
        nb ^= 1;
        for (int m = 1; m < p; ++m) {
          if (m == n) continue;
          ttm(cur, prod_range(dims, 0, m), dims[m], prod_range(dims, m + 1, p),
                       Fp(lo.A[i]) + A_off(i, m), dims[m], 1, rq[m], bufs[nb], false);
          dims[m] = rq[m];
          cur = bufs[nb];
          nb ^= 1;
        }
        // W_i^(n) into the stack Wst (ka x sr_n x kb) at mode-n rows roff_i
        const int ri = dims[n];
        const int64_t rb = int64_t(ri) * kb;
        const int srn = lo.sr[n];
        for (int64_t e = tid; e < ka * rb; e += nt) {
          const int64_t x = e / rb, jy = e - x * rb;
          Wst[(x * srn + sh.roff[n][i]) * kb + jy] = cur[e];
        }
        __syncthreads();
      }
      // K_n = sum_i W_i^(n) x_n C_i: one product over the stacked mode
      ttm(Wst, ka, lo.sr[n], kb, Fp(lo.C[n]), lo.sr[n], 1, q, K, false);
      with_eig_buf(q, [&](double* Wn, double* Wv) {
        gram(K, ka, q, kb, Wn, q);
        clk.mark(5);
        sweep_eig(n, Wn, Wv, q, rq[n]);
      });
      update_A(n);
      clk.mark(6);
    }
    // core update: G = Z^(p) x_p U^(p)T, here K_p x_p P_p^T
    {
      const int q = sh.q[p - 1];
      ttm(K, prod_range(rq, 0, p - 1), q, 1, Fp(lo.Pf[p - 1]), 1, rq[p - 1], rq[p - 1], G, false);
      const int64_t gel = prod_range(rq, 0, p);
      double part = 0.0;
      for (int64_t e = tid; e < gel; e += nt) part += double(G[e]) * double(G[e]);
      g2 = block_sum(part, red);
    }
    fit = ny2 > 0.0 ? 1.0 - sqrt(fmax(0.0, ny2 - g2)) / sqrt(ny2) : 1.0;
    sweeps = it;
    clk.mark(5);
    if (it >= 2 && fabs(fit - fit_prev) < tol) {
      conv = 1;
      break;
    }
    fit_prev = fit;
  }

  // ---- write the result ----------------------------------------------------------
  // (FP64 products on the matrix cores, FP32 stores)
  // U^(n) = B P_n (= V_cat F_n P_n on the basis route)
  for (int n = 1; n < p; ++n) {
    const int64_t Dn = st.D[n];
    const int r_out = rq[n];
    const double* P = Dp(lo.Pd[n]);
    float* out = job.out_fac[n];
    if (sh.basis[n]) {
      const int sr = lo.sr[n], q = sh.q[n];
      const double* Fn = Dp(lo.Fn[n]);
      double* Fh = Dp(lo.Fh[n]);
      gemm_f64(sr, r_out, q, [&](int c, int dd) { return Fn[c * sr + dd]; },
               [&](int dd, int j) { return P[dd * r_out + j]; },
               [&](int c, int j, double v) { Fh[c * r_out + j] = v; });
      gemm_f64_rows<4>(int(Dn), r_out, sr, [&](int dd, int c) { return vcat(n, dd, c); },
                       [&](int c, int j) { return Fh[c * r_out + j]; },
                       [&](int dd, int j, double v) { out[int64_t(dd) * r_out + j] = float(v); });
    } else {
      for (int64_t e = tid; e < Dn * r_out; e += nt) out[e] = float(P[e]);
    }
  }
  // U^(1) rows: block i = V~_i^(1) P_i, V~_i^(1) = rows F_i on a partial hit
  {
    const double* P0 = Dp(lo.Pd[0]);
    const int r0 = rq[0];
    int64_t t = 0;
    for (int i = 0; i < s; ++i) {
      const Hit h = hits[i];
      const int lev = h.level;
      const int k = st.rk[lev][0];
      const int kp = sh.kp[i];
      double* F0 = Dp(lo.F0[i]);  // k x r0
      const double* Pi = P0 + int64_t(sh.koff[i]) * r0;
      if (h.partial) {
        const double* Fi = Dp(lo.F[i]);
        gemm_f64(k, r0, kp, [&](int c, int m) { return Fi[c * k + m]; }, [&](int m, int j) { return Pi[m * r0 + j]; },
                 [&](int c, int j, double v) { F0[c * r0 + j] = v; });
      } else {
        for (int e = tid; e < k * r0; e += nt) F0[e] = Pi[e];
        __syncthreads();
      }
      const float* V = st.plane[lev] + ((h.index << lev) * st.ell + h.a) * k;
      float* out = job.out_fac[0] + t * r0;
      if (k <= 16 && r0 <= 16)
        gemm_f64_tall<8>(int(h.l), r0, k, [&](int row, int c) { return V[int64_t(row) * k + c]; },
                         [&](int c, int j) { return F0[c * r0 + j]; },
                         [&](int row, int j, double v) { out[int64_t(row) * r0 + j] = float(v); });
      else
        gemm_f64_rows<4>(int(h.l), r0, k, [&](int row, int c) { return V[int64_t(row) * k + c]; },
                         [&](int c, int j) { return F0[c * r0 + j]; },
                         [&](int row, int j, double v) { out[int64_t(row) * r0 + j] = float(v); });
      t += h.l;
    }
  }
  // final core in FP64: G = sum_i H~_i x_1 P_i^T x_{n>=2} (P_n^T C_i), and
  // the model error |Y~|^2 - |G|^2 from it
  {
    const int64_t gel = prod_range(rq, 0, p);
    double* G64 = Dp(lo.G64);
    double* D1 = Dp(lo.D1);
    double* D2 = Dp(lo.D2);
    const double* P0 = Dp(lo.Pd[0]);
    // [A64_1 .. A64_s] = P_n^T C^(n) for every mode
    for (int n = 1; n < p; ++n) {
      const int q = sh.q[n], sr = lo.sr[n], r_out = rq[n];
      const double* P = Dp(lo.Pd[n]);
      const double* C = Dp(lo.C64[n]);
      gemm_f64(r_out, sr, q, [&](int c, int dd) { return P[dd * r_out + c]; },
               [&](int dd, int col) { return C[int64_t(dd) * sr + col]; },
               [&](int c, int col, double v) {
                 const int i = hit_of_col(n, col);
                 const int r = st.rk[hits[i].level][n];
                 Dp(lo.A64[i])[A_off(i, n) + int64_t(c) * r + (col - sh.roff[n][i])] = v;
               });
    }
    for (int i = 0; i < s; ++i) {
      int32_t dims[PM];
      dims[0] = sh.kp[i];
      for (int m = 1; m < p; ++m) dims[m] = st.rk[hits[i].level][m];
      mode_product_f64<float>(core_of(i), 1, dims[0], prod_range(dims, 1, p), P0 + int64_t(sh.koff[i]) * rq[0], 1,
                              rq[0], rq[0], D1, false);
      dims[0] = rq[0];
      const double* cur = D1;
      double* bufs[2] = {D2, D1};
      int nb = 0;
      for (int n = 1; n < p; ++n) {
        double* out = (n == p - 1) ? G64 : bufs[nb];
        mode_product_f64<double>(cur, prod_range(dims, 0, n), dims[n], prod_range(dims, n + 1, p),
                                 Dp(lo.A64[i]) + A_off(i, n), dims[n], 1, rq[n], out, n == p - 1 && i > 0);
        dims[n] = rq[n];
        cur = out;
        nb ^= 1;
      }
    }
    double part = 0.0;
    for (int64_t e = tid; e < gel; e += nt) {
      part += G64[e] * G64[e];
      job.out_core[e] = float(G64[e]);
    }
    g2 = block_sum(part, red);
  }
  if (tid == 0 && job.stats) {
    job.stats[STAT_STATUS] = 0.0;
    job.stats[STAT_FIT] = fit;
    job.stats[STAT_ERR] = ny2 > 0.0 ? sqrt(fmax(0.0, ny2 - g2)) / sqrt(ny2) : 0.0;
    job.stats[STAT_NORM] = sqrt(ny2);
    job.stats[STAT_SWEEPS] = double(sweeps);
    job.stats[STAT_CONV] = double(conv);
    job.stats[STAT_HITS] = double(s);
  }
  clk.mark(7);
  clk.store(job.stats);
  if (tid == 0 && job.stats) {
    job.stats[STAT_EIG + 0] = double(ec.calls);
    job.stats[STAT_EIG + 1] = double(ec.sweeps);
    job.stats[STAT_EIG + 2] = double(ec.values_ticks) * 0.01;
    job.stats[STAT_EIG + 3] = double(ec.tail_ticks) * 0.01;
    job.stats[STAT_EIG_FALLBACK] = double(ec.fallbacks);
    job.stats[STAT_EIG_TRI] = double(ec.tri_ticks) * 0.01;
    job.stats[STAT_EIG_INVIT] = double(ec.invit_ticks) * 0.01;
    job.stats[STAT_EIG_WARM] = double(ec.warm);
    job.stats[STAT_EIG_WARM_FAIL] = double(ec.warm_fail);
    job.stats[STAT_EIG_WARM_STEPS] = double(ec.warm_steps);
    job.stats[STAT_EIG_WARM_US] = double(ec.warm_ticks) * 0.01;
    job.stats[STAT_EIG_WARM_RR_US] = double(ec.warm_rr_ticks) * 0.01;
  }
}

// One wavefront per job for jobs whose eigenproblems are small; two or four
// wavefronts for jobs with large ones (more lanes per rotation pair and per
// contraction shorten their latency, which bounds a batch's completion).
// A query job first runs Recall (Alg. "recall") on its own range and
// snapshot, into LDS, and publishes the hits to its slots of args.hits.
// With args.queue set the launch is persistent: each workgroup takes jobs
// from the queue counter (heaviest first, as the host sorted them) until it
// runs past n_jobs, so every workgroup reaches the exit.
// Register budget: at most 256 VGPRs, so that two wavefronts share a SIMD
// (one job's latency hides behind another's).
// Claim the next published job of the ring (thread 0): its sequence number,
// or -1 when the workgroup should stop: stop set, no job published for
// idle_ticks, or the launch older than life_ticks (then it ends even with
// jobs waiting, so that the class's hardware queue also serves the work of
// other streams; the scheduler relaunches at once).
__device__ __forceinline__ int64_t ring_claim(const StitchRing& r, uint64_t t_launch) {
  const uint64_t t_idle = wall_clock64();
  for (;;) {
    const uint64_t now = wall_clock64();
    if (now - t_launch > r.life_ticks) return -1;
    const int64_t tail = __hip_atomic_load(&r.hdr->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    int64_t h = __hip_atomic_load(r.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (h < tail) {
      if (__hip_atomic_compare_exchange_strong(r.head, &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT))
        return h;
      continue;
    }
    if (__hip_atomic_load(&r.hdr->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) || now - t_idle > r.idle_ticks)
      return -1;
    __builtin_amdgcn_s_sleep(16);
  }
}

template <int NTT, int PM>
__global__ __launch_bounds__(NTT, 2) void stitch_kernel(StitchArgs args) {
  extern __shared__ double lds[];
  __shared__ StitchShared<PM> sh;
  __shared__ Hit qh[MAXHITS];
  __shared__ int next_job;
  __shared__ int n_rec;
  __shared__ Job rjob;       // the job's descriptor (a ring job's copied from host memory)
  __shared__ int64_t rseq;
  const StoreView& st = *args.st;
  const bool ring = args.ring.hdr != nullptr;
  const uint64_t t_launch = wall_clock64();
  int jn = blockIdx.x;
  int64_t seq = -1;
  for (;;) {
    if (ring) {
      if (threadIdx.x == 0) {
        rseq = ring_claim(args.ring, t_launch);
        if (rseq >= 0) rjob = args.ring.jobs[rseq % args.ring.hdr->slots];
      }
      __syncthreads();
      seq = rseq;
      if (seq < 0) break;
    } else if (args.queue) {
      if (threadIdx.x == 0) next_job = atomicAdd(args.queue, 1);
      __syncthreads();
      jn = next_job;
      __syncthreads();
    }
    if (!ring && jn >= args.n_jobs) break;
    if (!ring) {  // the job's descriptor to LDS, as a ring job's
      if (threadIdx.x == 0) rjob = args.jobs[jn];
      __syncthreads();
    }
    const Job& job = rjob;
    // a ring job's statistics and outputs become visible to the host before
    // its completion word does
    auto ring_done = [&]() {
      if (!ring) return;
      __threadfence_system();
      __syncthreads();
      if (threadIdx.x == 0)
        __hip_atomic_store(&args.ring.done[seq % args.ring.hdr->slots], seq + 1, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      __syncthreads();  // rjob and rseq are rewritten by the next claim
    };
    if (st.p > PM) {  // launched with the wrong instantiation: refuse the job
      if (threadIdx.x == 0 && job.stats) job.stats[STAT_STATUS] = 3.0;
      ring_done();
      if (!args.queue && !ring) break;
      continue;
    }
    // the job's hits go to LDS: a query's from its own Recall (published to
    // its slots of args.hits), a merge's two children from args.hits
    if (threadIdx.x == 0) {
      int n = job.s;
      if (job.kind == 0) {
        n = recall_with_stack(job.ts, job.ts + job.L, job.Tb, st.ell, args.theta_num, args.theta_den, qh, MAXHITS,
                              sh.recall_stack);
        if (n == job.s)
          for (int i = 0; i < n; ++i) args.hits[job.hit0 + i] = qh[i];
      } else {
        for (int i = 0; i < n && i < MAXHITS; ++i) qh[i] = args.hits[job.hit0 + i];
      }
      n_rec = n;
    }
    __syncthreads();
    if (n_rec != job.s) {
      if (threadIdx.x == 0 && job.stats) {
        job.stats[STAT_STATUS] = 1.0;
        job.stats[STAT_HITS] = double(n_rec);
      }
      ring_done();
      if (!args.queue && !ring) break;
      continue;
    }
    const Hit* hits = qh;
    const uint64_t t_begin = wall_clock64();
    stitch_one(st, job, hits, args.ws + job.ws_off, args.n_lds, args.lds_doubles, args.basis_pct,
               job.kind == 1 ? args.merge_max_iter : args.max_iter, job.kind == 1 ? args.merge_tol : args.tol,
               job.kind == 1 ? args.merge_bf16 != 0 : args.bf16 != 0, sh, lds);
    if (threadIdx.x == 0 && job.stats) {
      job.stats[STAT_T0] = double(t_begin);
      job.stats[STAT_T1] = double(wall_clock64());
    }
    ring_done();
    if (!args.queue && !ring) break;
  }
}

}  // namespace tk
