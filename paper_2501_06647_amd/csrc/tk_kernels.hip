// Stitch and leaf kernels (gfx950).
//
// stitch_kernel: one workgroup per job.  A job is a range query (Sec. 6.1:
// Recall's hits -> partial-hit trims, Eq. "partial-tucker" -> Alg. "stitch")
// or the merge of two children when a node completes (Alg. "insert").
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
// FP64 Jacobi eigensolver.  Partial hits are trimmed through the Gram of the
// sliced rows: rows = Q~ R~ with R~ = Lambda^{1/2} E^T, Q~ = rows E Lambda^{-1/2}
// (an exact orthonormal factorisation, equivalent to the QR of
// Eq. "partial-tucker" up to a rotation of the piece's core).  Full-size
// factors are formed once, in FP64, when the result is written.
//
// leaf_kernel: one workgroup per leaf block; Tucker-ALS (Sec. 2) of the raw
// ell x D_2 x ... x D_p block with HOSVD initialisation.
#include "tk_device.hpp"
#include "tk_internal.hpp"

namespace tk {

// Flat copy with a grid-stride-free workgroup loop.
__device__ inline void wg_copy(float* dst, const float* src, int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

__device__ inline int64_t prod_range(const int32_t* d, int lo, int hi) {
  int64_t r = 1;
  for (int m = lo; m < hi; ++m) r *= d[m];
  return r;
}

// Phase timer: thread 0 accumulates the 100 MHz wall clock between marks.
struct PhaseClock {
  uint64_t last = 0;
  uint64_t acc[STAT_NPHASE] = {0, 0, 0, 0, 0, 0, 0, 0};
  __device__ void start() {
    if (threadIdx.x == 0) last = wall_clock64();
  }
  __device__ void mark(int ph) {
    if (threadIdx.x == 0) {
      const uint64_t now = wall_clock64();
      acc[ph] += now - last;
      last = now;
    }
  }
  __device__ void store(double* stats) const {
    if (threadIdx.x == 0 && stats)
      for (int i = 0; i < STAT_NPHASE; ++i) stats[STAT_PHASE + i] = double(acc[i]) * 0.01;
  }
};

struct StitchShared {
  StitchLayout lo;
  Hit hits[MAXHITS];
  int32_t kp[MAXHITS];          // temporal rank of each piece after its trim
  int32_t koff[MAXHITS + 1];    // offsets of the pieces in the stacked temporal coordinates
  int32_t roff[MAXP][MAXHITS + 1];  // offsets of the pieces' columns in C^(n)
  int32_t q[MAXP];              // size of the reduced coordinates of mode n
  int32_t basis[MAXP];          // 1: C^(n) = Lambda^{1/2} E^T; 0: C^(n) = V~
  double red[8];
  double small[1024];           // mode Gram of one core (r <= 32)
};

// Eigen workspace: LDS when the problem fits, else the job's global buffer.
__device__ inline double* eig_buf(int n, int n_lds, double* lds, char* ws, const StitchLayout& lo) {
  if (n <= n_lds) return lds;
  return reinterpret_cast<double*>(ws + lo.EIG);
}

__device__ void stitch_one(const StoreView& st, const Job& job, const Hit* ghits, char* ws,
                           int n_lds, int max_iter, double tol, StitchShared& sh, double* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int p = st.p;
  const int s = job.s;
  for (int i = tid; i < s; i += nt) sh.hits[i] = ghits[job.hit0 + i];
  __syncthreads();
  const int32_t* rq = job.rq;

  // One entire hit: the range is a stored node; return it verbatim.
  if (s == 1 && !sh.hits[0].partial) {
    const Hit h = sh.hits[0];
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
    }
    return;
  }

  PhaseClock clk;
  EigCounters ec;
  clk.start();
  if (tid == 0) stitch_layout(st, sh.hits, s, rq, n_lds, &sh.lo);
  __syncthreads();
  const StitchLayout& lo = sh.lo;
  double* red = sh.red;
  auto Fp = [&](int64_t off) { return reinterpret_cast<float*>(ws + off); };
  auto Dp = [&](int64_t off) { return reinterpret_cast<double*>(ws + off); };
  auto Fp64 = Dp;

  // ---- trims (Eq. "partial-tucker") and |Y~|^2 ------------------------------
  double ny2 = 0.0;
  for (int i = 0; i < s; ++i) {
    const Hit h = sh.hits[i];
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
    const float* V = st.plane[lev] + ((h.index << lev) * st.ell + h.a) * k;
    double* Wm = eig_buf(k, n_lds, lds, ws, lo);
    gram_mode<double>(V, h.l, k, 1, Wm, k);
    double* E = Dp(lo.F[i]);  // k x k, becomes F_i = E Lambda^{-1/2}
    const double* lam = eig_top(Wm, k, k, E, k, red, 1e-12, &ec);
    int kp = 0;
    for (int j = 0; j < k; ++j)
      if (lam[j] > 1e-12) kp = j + 1;
    // R~ (kp x k) in FP32 into T1, then H~ = R~ x_1 H
    float* Rt = Fp(lo.T1);
    for (int e = tid; e < kp * k; e += nt) {
      const int j = e / k, c = e % k;
      Rt[e] = float(sqrt(lam[j]) * E[c * k + j]);
    }
    __syncthreads();
    float* Ht = Fp(lo.Ht[i]);
    mode_product(H, 1, k, R, Rt, k, 1, kp, Ht, false);
    for (int e = tid; e < k * kp; e += nt) {
      const int c = e / kp, j = e % kp;
      E[c * k + j] /= sqrt(lam[j]);
    }
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
      for (int i = 0; i < s; ++i) sh.roff[n][i + 1] = sh.roff[n][i] + st.rk[sh.hits[i].level][n];
    }
  }
  __syncthreads();
  auto core_of = [&](int i) -> const float* {
    const Hit& h = sh.hits[i];
    return h.partial ? Fp(lo.Ht[i]) : st.core[h.level] + h.index * st.core_elems[h.level];
  };
  auto fac_of = [&](int i, int n) -> const float* {
    const Hit& h = sh.hits[i];
    return st.fac[h.level][n] + h.index * fac_elems(st, h.level, n);
  };
  auto A_of = [&](int i, int n) -> float* {  // U^(n)T V~_i^(n) = P_n^T C_i, rq_n x r_i^(n)
    int64_t off = 0;
    for (int m = 1; m < n; ++m) off += int64_t(rq[m]) * st.rk[sh.hits[i].level][m];
    return Fp(lo.A[i]) + off;
  };

  // ---- orthonormal bases of the non-temporal spans -----------------------------
  for (int n = 1; n < p; ++n) {
    const int sr = lo.sr[n];
    const int64_t Dn = st.D[n];
    float* C = Fp(lo.C[n]);  // q x sr, leading dimension sr
    int use_basis = 0;
    if (sr < Dn) {
      double* Wm = eig_buf(sr, n_lds, lds, ws, lo);
      for (int e = tid; e < sr * sr; e += nt) {
        const int x = e / sr, y = e % sr;
        if (y < x) continue;
        int ix = 0, iy = 0;
        while (x >= sh.roff[n][ix + 1]) ++ix;
        while (y >= sh.roff[n][iy + 1]) ++iy;
        const int rx = st.rk[sh.hits[ix].level][n], ry = st.rk[sh.hits[iy].level][n];
        const float* Vx = fac_of(ix, n) + (x - sh.roff[n][ix]);
        const float* Vy = fac_of(iy, n) + (y - sh.roff[n][iy]);
        double acc = 0.0;
        for (int64_t d = 0; d < Dn; ++d) acc += double(Vx[d * rx]) * double(Vy[d * ry]);
        Wm[x * sr + y] = acc;
        Wm[y * sr + x] = acc;
      }
      __syncthreads();
      double* E = Dp(lo.Fn[n]);  // sr x sr; becomes F_n = E Lambda^{-1/2}
      const double* lam = eig_top(Wm, sr, sr, E, sr, red, 1e-11, &ec);
      int q = 0;
      const double lmax = lam[0];
      for (int j = 0; j < sr; ++j)
        if (lam[j] > 1e-11 * lmax) q = j + 1;
      if (q >= rq[n]) {
        use_basis = 1;
        for (int e = tid; e < q * sr; e += nt) {
          const int d = e / sr, c = e % sr;
          const double cv = sqrt(lam[d]) * E[c * sr + d];
          C[d * sr + c] = float(cv);
          Fp64(lo.C64[n])[d * sr + c] = cv;
        }
        __syncthreads();
        for (int e = tid; e < sr * q; e += nt) {
          const int c = e / q, d = e % q;
          E[c * sr + d] /= sqrt(lam[d]);
        }
        if (tid == 0) sh.q[n] = q;
      }
    }
    if (!use_basis) {
      for (int64_t e = tid; e < Dn * sr; e += nt) {
        const int64_t d = e / sr;
        const int c = int(e % sr);
        int i = 0;
        while (c >= sh.roff[n][i + 1]) ++i;
        const int r = st.rk[sh.hits[i].level][n];
        C[e] = fac_of(i, n)[d * r + (c - sh.roff[n][i])];
        Fp64(lo.C64[n])[e] = double(C[e]);
      }
      if (tid == 0) sh.q[n] = int32_t(Dn);
    }
    if (tid == 0) sh.basis[n] = use_basis;
    __syncthreads();
  }

  clk.mark(1);
  // P_n^T C_i for every piece (mode n >= 1)
  auto update_A = [&](int n) {
    const int q = sh.q[n], sr = lo.sr[n], r_out = rq[n];
    const double* P = Dp(lo.Pd[n]);
    const float* C = Fp(lo.C[n]);
    for (int i = 0; i < s; ++i) {
      const int r = st.rk[sh.hits[i].level][n];
      float* A = A_of(i, n);
      const int c0 = sh.roff[n][i];
      for (int e = tid; e < r_out * r; e += nt) {
        const int c = e / r, j = e % r;
        double acc = 0.0;
        for (int d = 0; d < q; ++d) acc += P[d * r_out + c] * double(C[d * sr + c0 + j]);
        A[e] = float(acc);
      }
    }
    float* Pf = Fp(lo.Pf[n]);
    for (int e = tid; e < q * r_out; e += nt) Pf[e] = float(P[e]);
    __syncthreads();
  };

  // ---- HOSVD initialisation of U^(2..p) (Gram of Y~ in reduced coordinates)
  for (int n = 1; n < p; ++n) {
    const int q = sh.q[n], sr = lo.sr[n];
    double* Wm = eig_buf(q, n_lds, lds, ws, lo);
    for (int e = tid; e < q * q; e += nt) Wm[e] = 0.0;
    __syncthreads();
    for (int i = 0; i < s; ++i) {
      const int lev = sh.hits[i].level;
      const int r = st.rk[lev][n];
      int32_t dims[MAXP];
      dims[0] = sh.kp[i];
      for (int m = 1; m < p; ++m) dims[m] = st.rk[lev][m];
      gram_mode<double>(core_of(i), prod_range(dims, 0, n), r, prod_range(dims, n + 1, p), sh.small, r);
      double* T = Dp(lo.D1);  // C_i S_i, q x r
      const double* C64 = Dp(lo.C64[n]);
      const int c0 = sh.roff[n][i];
      for (int e = tid; e < q * r; e += nt) {
        const int d = e / r, j = e % r;
        double acc = 0.0;
        for (int c = 0; c < r; ++c) acc += C64[d * sr + c0 + c] * sh.small[c * r + j];
        T[e] = acc;
      }
      __syncthreads();
      for (int e = tid; e < q * q; e += nt) {
        const int d = e / q, d2 = e % q;
        double acc = 0.0;
        for (int j = 0; j < r; ++j) acc += T[d * r + j] * C64[d2 * sr + c0 + j];
        Wm[e] += acc;
      }
      __syncthreads();
    }
    eig_top(Wm, q, rq[n], Dp(lo.Pd[n]), rq[n], red, 0.0, &ec);
    update_A(n);
  }

  clk.mark(2);
  // ---- ALS sweeps (Alg. "stitch") ---------------------------------------------
  int64_t Rhat[MAXP];
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
    // temporal mode: M = [mat_1(H~_i x_{m>=2} A_i^(m))]_i, P_0 = leading eigvecs of M M^T
    float* M = Fp(lo.M);
    for (int i = 0; i < s; ++i) {
      const int lev = sh.hits[i].level;
      int32_t dims[MAXP];
      dims[0] = sh.kp[i];
      for (int m = 1; m < p; ++m) dims[m] = st.rk[lev][m];
      const float* cur = core_of(i);
      for (int n = 1; n < p; ++n) {
        float* out = (n == p - 1) ? M + int64_t(sh.koff[i]) * Rhat[0] : ((n & 1) ? T1 : T2);
        mode_product(cur, prod_range(dims, 0, n), dims[n], prod_range(dims, n + 1, p), A_of(i, n),
                     dims[n], 1, rq[n], out, false);
        dims[n] = rq[n];
        cur = out;
      }
    }
    const int sk = sh.koff[s];
    double* Wm = eig_buf(sk, n_lds, lds, ws, lo);
    gram_mode<double>(M, 1, sk, Rhat[0], Wm, sk);
    clk.mark(3);
    eig_top(Wm, sk, rq[0], Dp(lo.Pd[0]), rq[0], red, 0.0, &ec);
    clk.mark(4);
    float* P0f = Fp(lo.Pf[0]);
    {
      const double* P0 = Dp(lo.Pd[0]);
      for (int e = tid; e < sk * rq[0]; e += nt) P0f[e] = float(P0[e]);
      __syncthreads();
    }
    // non-temporal modes: K_n = sum_i W_i^(n) x_n C_i, P_n = leading eigvecs of its Gram
    float* K = Fp(lo.K);
    for (int n = 1; n < p; ++n) {
      const int q = sh.q[n];
      int32_t kd[MAXP];
      for (int m = 0; m < p; ++m) kd[m] = rq[m];
      kd[n] = q;
      const int64_t ka = prod_range(kd, 0, n), kb = prod_range(kd, n + 1, p);
      for (int i = 0; i < s; ++i) {
        const int lev = sh.hits[i].level;
        int32_t dims[MAXP];
        dims[0] = sh.kp[i];
        for (int m = 1; m < p; ++m) dims[m] = st.rk[lev][m];
        const float* cur = core_of(i);
        float* bufs[2] = {T1, T2};
        int nb = 0;
        // x_1 P_i^T : A(c, j) = P0[(koff_i + j) rq_0 + c]
        mode_product(cur, 1, dims[0], prod_range(dims, 1, p), P0f + int64_t(sh.koff[i]) * rq[0], 1,
                     rq[0], rq[0], bufs[nb], false);
        dims[0] = rq[0];
        cur = bufs[nb];
        nb ^= 1;
        for (int m = 1; m < p; ++m) {
          if (m == n) continue;
          mode_product(cur, prod_range(dims, 0, m), dims[m], prod_range(dims, m + 1, p), A_of(i, m),
                       dims[m], 1, rq[m], bufs[nb], false);
          dims[m] = rq[m];
          cur = bufs[nb];
          nb ^= 1;
        }
        // x_n C_i accumulated into K_n
        mode_product(cur, prod_range(dims, 0, n), dims[n], prod_range(dims, n + 1, p),
                     Fp(lo.C[n]) + sh.roff[n][i], lo.sr[n], 1, q, K, i > 0);
      }
      double* Wn = eig_buf(q, n_lds, lds, ws, lo);
      gram_mode<double>(K, ka, q, kb, Wn, q);
      clk.mark(5);
      eig_top(Wn, q, rq[n], Dp(lo.Pd[n]), rq[n], red, 0.0, &ec);
      update_A(n);
      clk.mark(6);
    }
    // core update: G = Z^(p) x_p U^(p)T, here K_p x_p P_p^T
    {
      const int q = sh.q[p - 1];
      mode_product(K, prod_range(rq, 0, p - 1), q, 1, Fp(lo.Pf[p - 1]), 1, rq[p - 1], rq[p - 1], G,
                   false);
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
  // U^(n) = B P_n (= V_cat F_n P_n on the basis route), formed in FP64
  for (int n = 1; n < p; ++n) {
    const int64_t Dn = st.D[n];
    const int r_out = rq[n];
    const double* P = Dp(lo.Pd[n]);
    float* out = job.out_fac[n];
    if (sh.basis[n]) {
      const int sr = lo.sr[n], q = sh.q[n];
      const double* Fn = Dp(lo.Fn[n]);
      double* Fh = Dp(lo.Fh[n]);
      for (int e = tid; e < sr * r_out; e += nt) {
        const int c = e / r_out, j = e % r_out;
        double acc = 0.0;
        for (int d = 0; d < q; ++d) acc += Fn[c * sr + d] * P[d * r_out + j];
        Fh[e] = acc;
      }
      __syncthreads();
      for (int64_t e = tid; e < Dn * r_out; e += nt) {
        const int64_t d = e / r_out;
        const int j = int(e % r_out);
        double acc = 0.0;
        for (int i = 0; i < s; ++i) {
          const int r = st.rk[sh.hits[i].level][n];
          const float* V = fac_of(i, n) + d * r;
          const double* f = Fh + int64_t(sh.roff[n][i]) * r_out + j;
          for (int c = 0; c < r; ++c) acc += double(V[c]) * f[int64_t(c) * r_out];
        }
        out[e] = float(acc);
      }
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
      const Hit h = sh.hits[i];
      const int lev = h.level;
      const int k = st.rk[lev][0];
      const int kp = sh.kp[i];
      double* F0 = Dp(lo.F0[i]);  // k x r0
      const double* Pi = P0 + int64_t(sh.koff[i]) * r0;
      if (h.partial) {
        const double* Fi = Dp(lo.F[i]);
        for (int e = tid; e < k * r0; e += nt) {
          const int c = e / r0, j = e % r0;
          double acc = 0.0;
          for (int m = 0; m < kp; ++m) acc += Fi[c * k + m] * Pi[m * r0 + j];
          F0[e] = acc;
        }
      } else {
        for (int e = tid; e < k * r0; e += nt) F0[e] = Pi[e];
      }
      __syncthreads();
      const float* V = st.plane[lev] + ((h.index << lev) * st.ell + h.a) * k;
      float* out = job.out_fac[0] + t * r0;
      for (int64_t e = tid; e < h.l * r0; e += nt) {
        const int64_t row = e / r0;
        const int j = int(e % r0);
        double acc = 0.0;
        for (int c = 0; c < k; ++c) acc += double(V[row * k + c]) * F0[c * r0 + j];
        out[e] = float(acc);
      }
      t += h.l;
      __syncthreads();
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
    for (int i = 0; i < s; ++i) {
      // A64_i^(n) = P_n^T C_i in FP64
      for (int n = 1; n < p; ++n) {
        const int q = sh.q[n], sr = lo.sr[n], r_out = rq[n];
        const int r = st.rk[sh.hits[i].level][n];
        const double* P = Dp(lo.Pd[n]);
        const double* C = Dp(lo.C64[n]);
        double* A = Dp(lo.A64[i]);
        for (int m = 1; m < n; ++m) A += int64_t(rq[m]) * st.rk[sh.hits[i].level][m];
        const int c0 = sh.roff[n][i];
        for (int e = tid; e < r_out * r; e += nt) {
          const int c = e / r, j = e % r;
          double acc = 0.0;
          for (int d = 0; d < q; ++d) acc += P[d * r_out + c] * C[d * sr + c0 + j];
          A[e] = acc;
        }
      }
      __syncthreads();
      int32_t dims[MAXP];
      dims[0] = sh.kp[i];
      for (int m = 1; m < p; ++m) dims[m] = st.rk[sh.hits[i].level][m];
      mode_product_t<float, double, double, double>(core_of(i), 1, dims[0], prod_range(dims, 1, p),
                                                    P0 + int64_t(sh.koff[i]) * rq[0], 1, rq[0], rq[0],
                                                    p == 1 ? G64 : D1, false);
      dims[0] = rq[0];
      const double* cur = D1;
      double* bufs[2] = {D2, D1};
      int nb = 0;
      for (int n = 1; n < p; ++n) {
        const double* A = Dp(lo.A64[i]);
        for (int m = 1; m < n; ++m) A += int64_t(rq[m]) * st.rk[sh.hits[i].level][m];
        double* out = (n == p - 1) ? G64 : bufs[nb];
        mode_product_t<double, double, double, double>(cur, prod_range(dims, 0, n), dims[n],
                                                       prod_range(dims, n + 1, p), A, dims[n], 1, rq[n],
                                                       out, n == p - 1 && i > 0);
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
    job.stats[STAT_EIG + 2] = double(ec.jacobi_ticks) * 0.01;
    job.stats[STAT_EIG + 3] = double(ec.tail_ticks) * 0.01;
  }
}

__global__ __launch_bounds__(NT) void stitch_kernel(StitchArgs args) {
  extern __shared__ double lds[];
  __shared__ StitchShared sh;
  stitch_one(*args.st, args.jobs[blockIdx.x], args.hits, args.ws + args.jobs[blockIdx.x].ws_off,
             args.n_lds, args.jobs[blockIdx.x].kind == 1 ? args.merge_max_iter : args.max_iter,
             args.jobs[blockIdx.x].kind == 1 ? args.merge_tol : args.tol, sh, lds);
}

// ------------------------------------------------------------------------------
// Leaf: Tucker-ALS of one raw block (Sec. 2), HOSVD initialisation.
// ------------------------------------------------------------------------------
struct LeafShared {
  LeafLayout lo;
  double red[8];
  double coef[64];
};

// Leading r left singular vectors of mat_n(Y) for Y of shape dims, as an
// FP64 D_n x r matrix U (row-major): the eigenvectors of the smaller Gram.
__device__ void leading_left(const float* Y, const int32_t* dims, int p, int n, int r, double* U,
                             double* Vbuf, int n_lds, double* lds, char* ws, const LeafLayout& lo,
                             LeafShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t a = prod_range(dims, 0, n), b = prod_range(dims, n + 1, p);
  const int D = dims[n];
  const int64_t N = a * b;
  if (D <= N) {
    double* Wm = D <= n_lds ? lds : reinterpret_cast<double*>(ws + lo.EIG);
    gram_mode<double>(Y, a, D, b, Wm, D);
    eig_top(Wm, D, r, U, r, sh.red);
    return;
  }
  const int Ni = int(N);
  double* Wm = Ni <= n_lds ? lds : reinterpret_cast<double*>(ws + lo.EIG);
  gram_other(Y, a, D, b, Wm, Ni);
  const double* lam = eig_top(Wm, Ni, r, Vbuf, r, sh.red);
  for (int64_t e = tid; e < int64_t(D) * r; e += nt) {
    const int d = int(e / r), j = int(e % r);
    double acc = 0.0;
    for (int64_t c = 0; c < N; ++c) acc += double(Y[((c / b) * D + d) * b + (c % b)]) * Vbuf[c * r + j];
    const double sv = sqrt(lam[j]);
    U[e] = sv > 0.0 ? acc / sv : 0.0;
  }
  __syncthreads();
  orthonormalize(U, D, r, r, sh.coef, sh.red);
}

// Y = X x_m U_m^T over every mode m != skip, largest reduction first.
__device__ const float* project(const float* X, const int32_t* Dm, int p, int skip, float* const* Uf,
                                const int32_t* rq, float* T1, float* T2, int32_t* dims_out) {
  int32_t dims[MAXP];
  for (int m = 0; m < p; ++m) dims[m] = Dm[m];
  bool done[MAXP] = {false, false, false, false, false, false};
  const float* cur = X;
  float* bufs[2] = {T1, T2};
  int nb = 0;
  for (int step = 0; step < p; ++step) {
    int best = -1;
    double bestr = 0.0;
    for (int m = 0; m < p; ++m) {
      if (m == skip || done[m]) continue;
      const double ratio = double(Dm[m]) / double(rq[m]);
      if (best < 0 || ratio > bestr) {
        best = m;
        bestr = ratio;
      }
    }
    if (best < 0) break;
    done[best] = true;
    mode_product(cur, prod_range(dims, 0, best), dims[best], prod_range(dims, best + 1, p), Uf[best], 1,
                 rq[best], rq[best], bufs[nb], false);
    dims[best] = rq[best];
    cur = bufs[nb];
    nb ^= 1;
  }
  for (int m = 0; m < p; ++m) dims_out[m] = dims[m];
  return cur;
}

__global__ __launch_bounds__(NT) void leaf_kernel(LeafArgs args) {
  extern __shared__ double lds[];
  __shared__ LeafShared sh;
  const StoreView& st = *args.st;
  const LeafJob job = args.jobs[blockIdx.x];
  char* ws = args.ws + job.ws_off;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int p = st.p;
  if (tid == 0) leaf_layout(st, args.n_lds, &sh.lo);
  __syncthreads();
  const LeafLayout& lo = sh.lo;
  const int32_t* rq = st.rk[0];
  int32_t Dm[MAXP];
  Dm[0] = int32_t(st.ell);
  for (int n = 1; n < p; ++n) Dm[n] = int32_t(st.D[n]);
  const int64_t size = prod_range(Dm, 0, p);
  double part = 0.0;
  for (int64_t e = tid; e < size; e += nt) part += double(job.X[e]) * double(job.X[e]);
  const double nx2 = block_sum(part, sh.red);

  float* Uf[MAXP];
  double* Ud[MAXP];
  for (int n = 0; n < p; ++n) {
    Uf[n] = reinterpret_cast<float*>(ws + lo.Uf[n]);
    Ud[n] = reinterpret_cast<double*>(ws + lo.Ud[n]);
  }
  double* Vbuf = reinterpret_cast<double*>(ws + lo.V);
  float* T1 = reinterpret_cast<float*>(ws + lo.T1);
  float* T2 = reinterpret_cast<float*>(ws + lo.T2);
  float* G = reinterpret_cast<float*>(ws + lo.G);
  auto to_f32 = [&](int n) {
    for (int64_t e = tid; e < int64_t(Dm[n]) * rq[n]; e += nt) Uf[n][e] = float(Ud[n][e]);
    __syncthreads();
  };
  // HOSVD: U^(n) = leading left singular vectors of mat_n(X)
  for (int n = 0; n < p; ++n) {
    leading_left(job.X, Dm, p, n, rq[n], Ud[n], Vbuf, args.n_lds, lds, ws, lo, sh);
    to_f32(n);
  }
  double fit = 0.0, fit_prev = 0.0, g2 = 0.0;
  int sweeps = 0, conv = 0;
  for (int it = 1; it <= args.max_iter; ++it) {
    for (int n = 0; n < p; ++n) {
      int32_t dims[MAXP];
      const float* Y = project(job.X, Dm, p, n, Uf, rq, T1, T2, dims);
      leading_left(Y, dims, p, n, rq[n], Ud[n], Vbuf, args.n_lds, lds, ws, lo, sh);
      to_f32(n);
    }
    int32_t dims[MAXP];
    const float* Gc = project(job.X, Dm, p, -1, Uf, rq, T1, T2, dims);
    const int64_t gel = prod_range(rq, 0, p);
    part = 0.0;
    for (int64_t e = tid; e < gel; e += nt) {
      G[e] = Gc[e];
      part += double(Gc[e]) * double(Gc[e]);
    }
    g2 = block_sum(part, sh.red);
    fit = nx2 > 0.0 ? 1.0 - sqrt(fmax(0.0, nx2 - g2)) / sqrt(nx2) : 1.0;
    sweeps = it;
    if (it >= 2 && fabs(fit - fit_prev) < args.tol) {
      conv = 1;
      break;
    }
    fit_prev = fit;
  }
  // store the leaf: core, non-temporal factors, temporal rows
  const int64_t b = job.block;
  wg_copy(st.core[0] + b * st.core_elems[0], G, st.core_elems[0]);
  for (int n = 1; n < p; ++n) wg_copy(st.fac[0][n] + b * fac_elems(st, 0, n), Uf[n], fac_elems(st, 0, n));
  wg_copy(st.plane[0] + b * st.ell * rq[0], Uf[0], st.ell * rq[0]);
  if (tid == 0 && job.stats) {
    job.stats[STAT_FIT] = fit;
    job.stats[STAT_ERR] = nx2 > 0.0 ? sqrt(fmax(0.0, nx2 - g2)) / sqrt(nx2) : 0.0;
    job.stats[STAT_NORM] = sqrt(nx2);
    job.stats[STAT_SWEEPS] = double(sweeps);
    job.stats[STAT_CONV] = double(conv);
    job.stats[STAT_HITS] = 0.0;
  }
}

// ------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------
hipError_t launch_stitch(const StitchArgs& a, int n_jobs, size_t lds_bytes, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(stitch_kernel, dim3(n_jobs), dim3(NT), lds_bytes, stream, a);
  return hipGetLastError();
}

hipError_t launch_leaf(const LeafArgs& a, int n_jobs, size_t lds_bytes, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(leaf_kernel, dim3(n_jobs), dim3(NT), lds_bytes, stream, a);
  return hipGetLastError();
}

hipError_t set_lds_limits(size_t stitch_bytes, size_t leaf_bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(stitch_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(stitch_bytes));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(leaf_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(leaf_bytes));
}

size_t stitch_static_lds() { return sizeof(StitchShared); }
size_t leaf_static_lds() { return sizeof(LeafShared); }

}  // namespace tk
