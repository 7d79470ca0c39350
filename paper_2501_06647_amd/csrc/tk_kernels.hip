// Leaf and raw-range kernels (gfx950) and the launchers of every kernel.
//
// leaf_kernel: one workgroup of four wavefronts per leaf block; Tucker-ALS
// (Sec. 2) of the raw ell x D_2 x ... x D_p block with HOSVD initialisation.
// raw_kernel: the same Tucker-ALS on one whole raw range per workgroup.
// The stitch kernel lives in tk_stitch.hpp; its instantiations are compiled
// in tk_stitch_inst.hip and reached through the entry points declared in
// tk_internal.hpp.
#include "tk_stitch.hpp"

namespace tk {

__global__ void reset_queue_kernel(int* queue, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) queue[i] = 0;
}

// The trim pass: one workgroup per chunk of a partial hit's rows, the
// chunk's FP64 Gram summed with every thread of the workgroup (a stitch job
// would stream these rows through one wavefront, a memory round trip per
// few rows).  The stitch kernel adds a hit's chunk Grams in chunk order.
constexpr int NT_TRIM = 256;
__global__ __launch_bounds__(NT_TRIM) void trim_gram_kernel(const TrimChunk* __restrict__ chunks, int64_t n) {
  __shared__ double part[NT_TRIM * 16];
  for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
    const TrimChunk ch = chunks[c];
    gram_rows(ch.V, ch.rows, ch.k, ch.out, ch.k, part, NT_TRIM);
  }
}

// ------------------------------------------------------------------------------
// Leaf: Tucker-ALS of one raw block (Sec. 2), HOSVD initialisation.
// ------------------------------------------------------------------------------
struct LeafShared {
  LeafLayout lo;
  double red[8];
  int redi[8];
  double coef[64];
  int flag;
};

// Leading r left singular vectors of mat_n(Y) for Y of shape dims, as an
// FP64 D_n x r matrix U (row-major): the eigenvectors of the smaller Gram.
__device__ __forceinline__ void leading_left(const float* Y, const int32_t* dims, int p, int n, int r, double* U, double* Vbuf,
                             int n_lds, double* lds, char* ws, const LeafLayout& lo, LeafShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t a = prod_range(dims, 0, n), b = prod_range(dims, n + 1, p);
  const int D = dims[n];
  const int64_t N = a * b;
  double* TMP = reinterpret_cast<double*>(ws + lo.TMP);
  if (D <= N) {
    double* Wm = D <= n_lds ? lds : reinterpret_cast<double*>(ws + lo.EIG);
    gram_mode_mfma(Y, a, D, b, Wm, D);
    eig_top(Wm, D, r, U, r, sh.red, TMP, nullptr, Wm + int64_t(D) * D);
    return;
  }
  const int Ni = int(N);
  double* Wm = Ni <= n_lds ? lds : reinterpret_cast<double*>(ws + lo.EIG);
  gram_other(Y, a, D, b, Wm, Ni);
  const double* lam = eig_top(Wm, Ni, r, Vbuf, r, sh.red, TMP, nullptr, Wm + int64_t(Ni) * Ni);
  for (int64_t e = tid; e < int64_t(D) * r; e += nt) {
    const int d = int(e / r), j = int(e % r);
    double acc = 0.0;
    for (int64_t c = 0; c < N; ++c) acc += double(Y[((c / b) * D + d) * b + (c % b)]) * Vbuf[c * r + j];
    const double sv = sqrt(lam[j]);
    U[e] = sv > 0.0 ? acc / sv : 0.0;
  }
  __syncthreads();
  orthonormalize(U, D, r, r, 1, sh.coef, sh.red, &sh.flag);
}

// Y = X x_m U_m^T over every mode m != skip, largest reduction first.
__device__ __forceinline__ const float* project(const float* X, const int32_t* Dm, int p, int skip, float* const* Uf,
                                const int32_t* rq, float* T1, float* T2, int32_t* dims_out) {
  int32_t dims[MAXP];
  for (int m = 0; m < p; ++m) dims[m] = Dm[m];
  bool done[MAXP] = {};
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

struct AlsResult {
  double fit, nx2, g2;
  int sweeps, conv;
};

// Tucker-ALS of an explicit block X (Dm[0] x ... x Dm[p-1], C order) at
// ranks rq: HOSVD init of U^(init_from..p-1), sweeps over every mode from
// mode 0, the fit stop rule of the stitch.  Leaves the FP32 factors in the
// workspace (lo.Uf) and the core in lo.G.
__device__ __forceinline__ AlsResult block_tucker_als(const float* X, const int32_t* Dm, const int32_t* rq, int p,
                                                      int init_from, int max_iter, double tol, int n_lds,
                                                      double* lds, char* ws, const LeafLayout& lo, LeafShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t size = prod_range(Dm, 0, p);
  double part = 0.0;
  for (int64_t e = tid; e < size; e += nt) part += double(X[e]) * double(X[e]);
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
  for (int n = init_from; n < p; ++n) {
    leading_left(X, Dm, p, n, rq[n], Ud[n], Vbuf, n_lds, lds, ws, lo, sh);
    to_f32(n);
  }
  double fit = 0.0, fit_prev = 0.0, g2 = 0.0;
  int sweeps = 0, conv = 0;
  for (int it = 1; it <= max_iter; ++it) {
    for (int n = 0; n < p; ++n) {
      int32_t dims[MAXP];
      const float* Y = project(X, Dm, p, n, Uf, rq, T1, T2, dims);
      leading_left(Y, dims, p, n, rq[n], Ud[n], Vbuf, n_lds, lds, ws, lo, sh);
      to_f32(n);
    }
    int32_t dims[MAXP];
    const float* Gc = project(X, Dm, p, -1, Uf, rq, T1, T2, dims);
    const int64_t gel = prod_range(rq, 0, p);
    part = 0.0;
    for (int64_t e = tid; e < gel; e += nt) {
      G[e] = Gc[e];
      part += double(Gc[e]) * double(Gc[e]);
    }
    g2 = block_sum(part, sh.red);
    fit = nx2 > 0.0 ? 1.0 - sqrt(fmax(0.0, nx2 - g2)) / sqrt(nx2) : 1.0;
    sweeps = it;
    if (it >= 2 && fabs(fit - fit_prev) < tol) {
      conv = 1;
      break;
    }
    fit_prev = fit;
  }
  return AlsResult{fit, nx2, g2, sweeps, conv};
}

__device__ __forceinline__ void als_stats(double* stats, const AlsResult& r) {
  if (threadIdx.x == 0 && stats) {
    stats[STAT_FIT] = r.fit;
    stats[STAT_ERR] = r.nx2 > 0.0 ? sqrt(fmax(0.0, r.nx2 - r.g2)) / sqrt(r.nx2) : 0.0;
    stats[STAT_NORM] = sqrt(r.nx2);
    stats[STAT_SWEEPS] = double(r.sweeps);
    stats[STAT_CONV] = double(r.conv);
    stats[STAT_HITS] = 0.0;
  }
}

// Start vectors of the subspace iteration: Wellons' lowbias32 integer hash
// of the element index, mapped to [-1, 1).
__device__ __forceinline__ double start_entry(uint32_t i) {
  uint32_t x = i + 0x9E3779B9u;
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return double(x) * (2.0 / 4294967296.0) - 1.0;
}

// The columns of E (n x k, element (i, j) at E[i * ld + j]) made orthonormal
// in place, left to right: Gram-Schmidt twice against the earlier columns.
// A column left with under 1e-10 of its norm lies in their span and is
// replaced by the first unit vector that does not, so the span stays
// k-dimensional (k <= n).  coef: k doubles.
__device__ __forceinline__ void orth_columns(double* E, int n, int k, int ld, double* coef, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nw = nt >> 6, w = tid >> 6, l = tid & 63;
  int cand = 0;
  for (int j = 0; j < k; ++j) {
    double part = 0.0;
    for (int i = tid; i < n; i += nt) part += E[int64_t(i) * ld + j] * E[int64_t(i) * ld + j];
    double n0 = sqrt(block_sum(part, red));
    for (;;) {
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        for (int c = w; c < j; c += nw) {
          double d = 0.0;
          for (int i = l; i < n; i += 64) d += E[int64_t(i) * ld + c] * E[int64_t(i) * ld + j];
          for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
          if (l == 0) coef[c] = d;
        }
        __syncthreads();
        for (int i = tid; i < n; i += nt) {
          double v = E[int64_t(i) * ld + j];
          for (int c = 0; c < j; ++c) v -= coef[c] * E[int64_t(i) * ld + c];
          E[int64_t(i) * ld + j] = v;
        }
        __syncthreads();
      }
      part = 0.0;
      for (int i = tid; i < n; i += nt) part += E[int64_t(i) * ld + j] * E[int64_t(i) * ld + j];
      const double n1 = sqrt(block_sum(part, red));
      if (n1 > 0.0 && n1 > 1e-10 * n0) {
        const double inv = 1.0 / n1;
        for (int i = tid; i < n; i += nt) E[int64_t(i) * ld + j] *= inv;
        __syncthreads();
        break;
      }
      if (cand >= n) {  // unreachable for k <= n: the unit vectors span everything
        for (int i = tid; i < n; i += nt) E[int64_t(i) * ld + j] = 0.0;
        __syncthreads();
        break;
      }
      for (int i = tid; i < n; i += nt) E[int64_t(i) * ld + j] = i == cand ? 1.0 : 0.0;
      ++cand;
      n0 = 1.0;
      __syncthreads();
    }
  }
}

// Leading r eigenpairs of S = A A^T for an n x m matrix A (a(i, c) returns
// A(i, c) in FP64), S never formed: block subspace iteration with b
// columns (b >= r + 8) and Rayleigh-Ritz (Golub & Van Loan, Sec. 8.2.4 and
// 8.1.4).  Each step: Z = A^T Q, Y = A Z = S Q; Q^T S Q = Z^T Z = W Theta W^T;
// Ritz vectors Q W, residuals S Q w_j - theta_j Q w_j = Y w_j - theta_j Q w_j.
// It stops once the leading r residuals are at most 1e-12 theta_1 (S's
// rounding level is near 1e-14 theta_1), or after max_it steps; otherwise
// Q becomes the orthonormalised Y W.  Writes U (n x r, the Ritz vectors),
// sv (sqrt(theta_j)), and Uo = A^T U diag(1/sv) (m x r, zero where sv is
// zero).  Returns the steps taken; *conv tells whether the test passed.
template <typename FA>
__device__ __forceinline__ int subspace_top(FA&& a, int n, int m, int r, int b, int max_it, int n_lds, double* lds,
                                            char* ws, const LeafLayout& lo, LeafShared& sh, double* U, double* Uo,
                                            double* sv, int* conv) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double* Q = reinterpret_cast<double*>(ws + lo.SQ);
  double* Y = reinterpret_cast<double*>(ws + lo.SY);
  double* QW = reinterpret_cast<double*>(ws + lo.SQW);
  double* YW = reinterpret_cast<double*>(ws + lo.SYW);
  double* Z = reinterpret_cast<double*>(ws + lo.SZ);
  double* W = reinterpret_cast<double*>(ws + lo.SW);
  double* TMP = reinterpret_cast<double*>(ws + lo.TMP);
  double* Bm = b <= n_lds ? lds : reinterpret_cast<double*>(ws + lo.EIG);
  for (int64_t e = tid; e < int64_t(n) * b; e += nt) Q[e] = start_entry(uint32_t(e));
  __syncthreads();
  orth_columns(Q, n, b, b, sh.coef, sh.red);
  int it = 0;
  *conv = 0;
  const double* lam = nullptr;
  for (;;) {
    ++it;
    gemm_f64(m, b, n, [&](int c, int i) { return a(i, c); }, [&](int i, int j) { return Q[int64_t(i) * b + j]; },
             [&](int c, int j, double v) { Z[int64_t(c) * b + j] = v; });
    gemm_f64(n, b, m, [&](int i, int c) { return a(i, c); }, [&](int c, int j) { return Z[int64_t(c) * b + j]; },
             [&](int i, int j, double v) { Y[int64_t(i) * b + j] = v; });
    gemm_f64(b, b, m, [&](int i, int c) { return Z[int64_t(c) * b + i]; },
             [&](int c, int j) { return Z[int64_t(c) * b + j]; }, [&](int i, int j, double v) { Bm[i * b + j] = v; });
    lam = eig_top(Bm, b, b, W, b, sh.red, TMP, nullptr, Bm + b * b);
    gemm_f64(n, b, b, [&](int i, int c) { return Q[int64_t(i) * b + c]; }, [&](int c, int j) { return W[c * b + j]; },
             [&](int i, int j, double v) { QW[int64_t(i) * b + j] = v; });
    gemm_f64(n, b, b, [&](int i, int c) { return Y[int64_t(i) * b + c]; }, [&](int c, int j) { return W[c * b + j]; },
             [&](int i, int j, double v) { YW[int64_t(i) * b + j] = v; });
    const double top = fmax(lam[0], 0.0);
    double worst = 0.0;
    for (int j = 0; j < r; ++j) {
      double part = 0.0;
      for (int i = tid; i < n; i += nt) {
        const double d = YW[int64_t(i) * b + j] - lam[j] * QW[int64_t(i) * b + j];
        part += d * d;
      }
      worst = fmax(worst, sqrt(block_sum(part, sh.red)));
    }
    if (worst <= 1e-12 * top) *conv = 1;
    if (*conv || it >= max_it) break;
    for (int64_t e = tid; e < int64_t(n) * b; e += nt) Q[e] = YW[e];
    __syncthreads();
    orth_columns(Q, n, b, b, sh.coef, sh.red);
  }
  for (int j = tid; j < r; j += nt) sv[j] = sqrt(fmax(lam[j], 0.0));
  for (int64_t e = tid; e < int64_t(n) * r; e += nt) U[e] = QW[(e / r) * b + e % r];
  __syncthreads();
  // A^T (Q W) = Z W
  gemm_f64(m, r, b, [&](int c, int k) { return Z[int64_t(c) * b + k]; }, [&](int k, int j) { return W[k * b + j]; },
           [&](int c, int j, double v) { Uo[int64_t(c) * r + j] = sv[j] > 0.0 ? v / sv[j] : 0.0; });
  return it;
}

// A leaf of one slice of a three-way series (leaf length 1): the temporal
// mode has length one, so its rank is one, the two other ranks are equal
// (r_2 <= r_1 r_3 and r_3 <= r_1 r_2), and Tucker-ALS on the slice reaches
// its truncated SVD: U^(2) the leading r left singular vectors of the D_2 x
// D_3 slice X, U^(3) = X^T U^(2) diag(1/s) (orthonormalised), the core
// U^(2)T X U^(3) (diagonal up to rounding), U^(1) = [1].  The leading
// singular vectors of the smaller side come from one eigensolve of its Gram
// (LEAF_SLICE_GRAM) or from subspace iteration on it (LEAF_SLICE_ITER);
// the other side's follow from them.  Leaves the results where
// block_tucker_als leaves them.
__device__ __forceinline__ AlsResult slice_svd(const float* X, const int32_t* Dm, int r, int max_it, int n_lds,
                                               double* lds, char* ws, const LeafLayout& lo, LeafShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int D2 = Dm[1], D3 = Dm[2];
  double part = 0.0;
  for (int64_t e = tid; e < int64_t(D2) * D3; e += nt) part += double(X[e]) * double(X[e]);
  const double nx2 = block_sum(part, sh.red);
  double* Ud1 = reinterpret_cast<double*>(ws + lo.Ud[1]);
  double* Ud2 = reinterpret_cast<double*>(ws + lo.Ud[2]);
  float* Uf0 = reinterpret_cast<float*>(ws + lo.Uf[0]);
  float* Uf1 = reinterpret_cast<float*>(ws + lo.Uf[1]);
  float* Uf2 = reinterpret_cast<float*>(ws + lo.Uf[2]);
  float* G = reinterpret_cast<float*>(ws + lo.G);
  double* TMP = reinterpret_cast<double*>(ws + lo.TMP);
  const bool left = D2 <= D3;
  const int n = left ? D2 : D3;   // the smaller side
  const int Do = left ? D3 : D2;  // the other side
  double* Us = left ? Ud1 : Ud2;  // leading singular vectors of the smaller side
  double* Uo = left ? Ud2 : Ud1;  // the other side's, X^T U / s or X V / s
  double* sv = sh.coef + 32;      // r <= 32 singular values
  int steps = 1, conv = 1;
  double* P;  // n x r scratch for the core
  if (lo.route == LEAF_SLICE_ITER) {
    const int b = slice_block(n, r);
    auto a = [&](int i, int c) {
      return left ? double(X[int64_t(i) * D3 + c]) : double(X[int64_t(c) * D3 + i]);
    };
    steps = subspace_top(a, n, Do, r, b, max_it, n_lds, lds, ws, lo, sh, Us, Uo, sv, &conv);
    P = reinterpret_cast<double*>(ws + lo.SY);  // n x b >= n x r
  } else {
    double* Wm = n <= n_lds ? lds : reinterpret_cast<double*>(ws + lo.EIG);
    if (left) gram_mode_mfma(X, 1, D2, D3, Wm, D2);
    else gram_other(X, 1, D2, D3, Wm, D3);
    const double* lam = eig_top(Wm, n, r, Us, r, sh.red, TMP, nullptr, Wm + int64_t(n) * n);
    for (int j = tid; j < r; j += nt) sv[j] = sqrt(fmax(lam[j], 0.0));
    __syncthreads();
    gemm_f64(Do, r, n,
             [&](int d, int c) { return left ? double(X[int64_t(c) * D3 + d]) : double(X[int64_t(d) * D3 + c]); },
             [&](int c, int j) { return Us[int64_t(c) * r + j]; },
             [&](int d, int j, double v) { Uo[int64_t(d) * r + j] = sv[j] > 0.0 ? v / sv[j] : 0.0; });
    P = TMP;  // eig_tmp_doubles(n) = n max(n, 128) >= n r
  }
  orthonormalize(Uo, Do, r, r, 1, sh.coef, sh.red, &sh.flag);
  // core G = U^(2)T X U^(3) (r x r) in FP64, through the smaller side's
  // n x r product
  if (left) {  // P = X U^(3) (D2 x r), G = U^(2)T P
    gemm_f64(D2, r, D3, [&](int i, int c) { return double(X[int64_t(i) * D3 + c]); },
             [&](int c, int j) { return Ud2[int64_t(c) * r + j]; }, [&](int i, int j, double v) { P[int64_t(i) * r + j] = v; });
    gemm_f64(r, r, D2, [&](int a, int i) { return Ud1[int64_t(i) * r + a]; },
             [&](int i, int j) { return P[int64_t(i) * r + j]; }, [&](int a, int j, double v) { G[a * r + j] = float(v); });
  } else {  // P = X^T U^(2) (D3 x r), G = P^T U^(3)
    gemm_f64(D3, r, D2, [&](int c, int i) { return double(X[int64_t(i) * D3 + c]); },
             [&](int i, int a) { return Ud1[int64_t(i) * r + a]; }, [&](int c, int a, double v) { P[int64_t(c) * r + a] = v; });
    gemm_f64(r, r, D3, [&](int a, int c) { return P[int64_t(c) * r + a]; },
             [&](int c, int j) { return Ud2[int64_t(c) * r + j]; }, [&](int a, int j, double v) { G[a * r + j] = float(v); });
  }
  part = 0.0;
  for (int e = tid; e < r * r; e += nt) part += double(G[e]) * double(G[e]);
  const double g2 = block_sum(part, sh.red);
  for (int64_t e = tid; e < int64_t(D2) * r; e += nt) Uf1[e] = float(Ud1[e]);
  for (int64_t e = tid; e < int64_t(D3) * r; e += nt) Uf2[e] = float(Ud2[e]);
  if (tid == 0) Uf0[0] = 1.0f;
  __syncthreads();
  const double fit = nx2 > 0.0 ? 1.0 - sqrt(fmax(0.0, nx2 - g2)) / sqrt(nx2) : 1.0;
  return AlsResult{fit, nx2, g2, steps, conv};
}

__global__ __launch_bounds__(NT_LEAF, 2) void leaf_kernel(LeafArgs args) {
  extern __shared__ double lds[];
  __shared__ LeafShared sh;
  const StoreView& st = *args.st;
  const LeafJob job = args.jobs[blockIdx.x];
  char* ws = args.ws + job.ws_off;
  const int p = st.p;
  if (threadIdx.x == 0) leaf_layout(st, args.n_lds, &sh.lo);
  __syncthreads();
  const LeafLayout& lo = sh.lo;
  const int32_t* rq = st.rk[0];
  int32_t Dm[MAXP];
  Dm[0] = int32_t(st.ell);
  for (int n = 1; n < p; ++n) Dm[n] = int32_t(st.D[n]);
  const bool svd = lo.route != LEAF_ALS;
  const AlsResult r = svd ? slice_svd(job.X, Dm, rq[1], kSliceIterMax, args.n_lds, lds, ws, lo, sh)
                          : block_tucker_als(job.X, Dm, rq, p, 0, args.max_iter, args.tol, args.n_lds, lds, ws, lo, sh);
  // store the leaf: core, non-temporal factors, temporal rows
  const int64_t b = job.block;
  const float* G = reinterpret_cast<const float*>(ws + lo.G);
  wg_copy(st.core[0] + b * st.core_elems[0], G, st.core_elems[0]);
  for (int n = 1; n < p; ++n)
    wg_copy(st.fac[0][n] + b * fac_elems(st, 0, n), reinterpret_cast<const float*>(ws + lo.Uf[n]),
            fac_elems(st, 0, n));
  wg_copy(st.plane[0] + b * st.ell * rq[0], reinterpret_cast<const float*>(ws + lo.Uf[0]), st.ell * rq[0]);
  als_stats(job.stats, r);
}

// Tucker-ALS from scratch on one raw range per workgroup (HOSVD of modes
// 1..p-1, sweeps from the temporal mode), written to the job's outputs.
__global__ __launch_bounds__(NT_LEAF, 2) void raw_kernel(RawArgs args) {
  extern __shared__ double lds[];
  __shared__ LeafShared sh;
  const RawJob job = args.jobs[blockIdx.x];
  char* ws = args.ws + job.ws_off;
  const int p = args.p;
  int32_t Dm[MAXP];
  Dm[0] = int32_t(job.L);
  for (int n = 1; n < p; ++n) Dm[n] = args.D[n];
  if (threadIdx.x == 0) raw_layout(p, Dm, job.rq, args.n_lds, &sh.lo);
  __syncthreads();
  const LeafLayout& lo = sh.lo;
  const AlsResult r = block_tucker_als(job.X, Dm, job.rq, p, 1, args.max_iter, args.tol, args.n_lds, lds, ws, lo, sh);
  wg_copy(job.out_core, reinterpret_cast<const float*>(ws + lo.G), prod_range(job.rq, 0, p));
  for (int n = 0; n < p; ++n)
    wg_copy(job.out_fac[n], reinterpret_cast<const float*>(ws + lo.Uf[n]), int64_t(Dm[n]) * job.rq[n]);
  als_stats(job.stats, r);
}

// ------------------------------------------------------------------------------
// Streaming Tucker-ALS on one long raw range: each pass gives every workgroup
// a span of consecutive slices, treated as a block of the range; what a
// pass reduces over time (a Gram, a mode-n product with U^(1)'s rows of the
// span) is linear in the slices, so the spans' partials sum to the range's.
// ------------------------------------------------------------------------------
__device__ __forceinline__ int64_t span_rows(const StreamArgs& a, int64_t t0) {
  const int64_t t1 = t0 + a.span < a.L ? t0 + a.span : a.L;
  return t1 - t0;
}

// Mode Gram G = sum over (x, y) of X[x][:][y] X[x][:][y]^T (q x q, FP64
// sums of exact FP32 products) for X viewed as (a, q, b) with b >= KC or
// b = 1, and q <= 16 SG_T: the columns stream through LDS in chunks of KC,
// loaded along the contiguous index (KC consecutive y, or for b = 1 the
// rows of KC consecutive x), and each wavefront keeps its 16 x 16 output
// tiles of the upper triangle in registers over all chunks
// (v_mfma_f64_16x16x4f64; operand layout that of gemm_f64).  Rows are
// padded by one float against bank conflicts.
constexpr int SG_KC = 32;  // columns per chunk
constexpr int SG_T = 8;    // q <= 128
constexpr int SG_SLOTS = 9;  // tiles per wavefront: 36 upper tiles over four wavefronts
__device__ __forceinline__ void gram_staged(const float* __restrict__ X, int64_t a, int q, int64_t b, double* G,
                                            float (*S)[SG_KC + 1]) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nw = nt >> 6, w = tid >> 6, l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  const int tq = (q + 15) >> 4;
  const int tiles = tq * (tq + 1) / 2;
  int TI[SG_SLOTS], TJ[SG_SLOTS];
  tk_d4 acc[SG_SLOTS];
#pragma unroll
  for (int sl = 0; sl < SG_SLOTS; ++sl) {
    int t = w + sl * nw, I = 0;
    while (t >= tq - I && I < tq) {  // upper-triangle tile t -> (I, J), I <= J
      t -= tq - I;
      ++I;
    }
    TI[sl] = I;
    TJ[sl] = I + t;
    acc[sl] = tk_d4{0.0, 0.0, 0.0, 0.0};
  }
  const bool rows = b == 1;  // chunks of KC consecutive x, each a contiguous row of q
  const int64_t nx = rows ? (a + SG_KC - 1) / SG_KC : a;
  for (int64_t x = 0; x < nx; ++x) {
    for (int64_t y0 = 0; y0 < b; y0 += SG_KC) {
      __syncthreads();  // the previous chunk is consumed
      if (rows) {
        const int64_t x0 = x * SG_KC;
        for (int e = tid; e < q * SG_KC; e += nt) {
          const int k = e / q, i = e % q;
          S[i][k] = x0 + k < a ? X[(x0 + k) * q + i] : 0.f;
        }
      } else {
        for (int e = tid; e < q * SG_KC; e += nt) {
          const int i = e / SG_KC, k = e % SG_KC;
          S[i][k] = y0 + k < b ? X[(x * q + i) * b + y0 + k] : 0.f;
        }
      }
      for (int e = q * SG_KC + tid; e < tq * 16 * SG_KC; e += nt) S[e / SG_KC][e % SG_KC] = 0.f;
      __syncthreads();
#pragma unroll
      for (int sl = 0; sl < SG_SLOTS; ++sl) {
        if (w + sl * nw < tiles) {
          const int ri = TI[sl] * 16 + lr, rj = TJ[sl] * 16 + lr;
#pragma unroll
          for (int kk = 0; kk < SG_KC / 4; ++kk) {
            const double av = double(S[ri][4 * kk + lk]);
            const double bv = double(S[rj][4 * kk + lk]);
            acc[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[sl], 0, 0, 0);
          }
        }
      }
    }
  }
#pragma unroll
  for (int sl = 0; sl < SG_SLOTS; ++sl) {
    if (w + sl * nw < tiles) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = TI[sl] * 16 + lk + 4 * v, j = TJ[sl] * 16 + lr;
        if (i < q && j < q) {
          G[int64_t(i) * q + j] = acc[sl][v];
          G[int64_t(j) * q + i] = acc[sl][v];
        }
      }
    }
  }
  __syncthreads();
}

// Partial Gram of mode a.skip (>= 1) of the span, and with a.nx2 its
// squared norm.
__global__ __launch_bounds__(NT_LEAF, 2) void stream_gram_kernel(StreamArgs a) {
  __shared__ double red[8];
  __shared__ float S[SG_T * 16][SG_KC + 1];
  const int64_t t0 = int64_t(blockIdx.x) * a.span;
  const int64_t rows = span_rows(a, t0);
  const float* Xc = a.X + t0 * a.slice;
  int32_t Dm[MAXP];
  Dm[0] = int32_t(rows);
  for (int m = 1; m < a.p; ++m) Dm[m] = a.D[m];
  const int n = a.skip;
  const int64_t ga = prod_range(Dm, 0, n), gb = prod_range(Dm, n + 1, a.p);
  double* G = a.part + int64_t(blockIdx.x) * a.part_elems;
  if ((gb >= SG_KC || gb == 1) && Dm[n] <= SG_T * 16 && blockDim.x == NT_LEAF)
    gram_staged(Xc, ga, Dm[n], gb, G, S);
  else
    gram_mode_mfma(Xc, ga, Dm[n], gb, G, Dm[n]);
  if (a.nx2) {
    double part = 0.0;
    for (int64_t e = threadIdx.x; e < rows * a.slice; e += blockDim.x) part += double(Xc[e]) * double(Xc[e]);
    part = block_sum(part, red);
    if (threadIdx.x == 0) a.nx2[blockIdx.x] = part;
  }
}

// The span projected on every mode but a.skip.  Temporal pass: its rows of
// Y = X x_{m>=2} U^(m)T and the partial Gram of those rows (R_1 x R_1).
// Mode n >= 1: X_span x_1 U^(1)[span]^T x_{m != n} U^(m)T, the span's share
// of the mode-n product, as FP64 into its partial slot.
__global__ __launch_bounds__(NT_LEAF, 2) void stream_project_kernel(StreamArgs a) {
  const int64_t t0 = int64_t(blockIdx.x) * a.span;
  const int64_t rows = span_rows(a, t0);
  int32_t Dm[MAXP];
  Dm[0] = int32_t(rows);
  for (int m = 1; m < a.p; ++m) Dm[m] = a.D[m];
  float* Uf[MAXP];
  for (int m = 0; m < a.p; ++m) Uf[m] = a.Uf[m];
  Uf[0] = a.Uf[0] + t0 * a.rq[0];
  char* ws = a.ws + int64_t(blockIdx.x) * a.ws_per;
  int32_t dims[MAXP];
  const float* Yc = project(a.X + t0 * a.slice, Dm, a.p, a.skip, Uf, a.rq, reinterpret_cast<float*>(ws),
                            reinterpret_cast<float*>(ws + a.t2_off), dims);
  const int64_t E = prod_range(dims, 0, a.p);
  double* part = a.part + int64_t(blockIdx.x) * a.part_elems;
  if (a.skip == 0) {
    const int64_t R1 = E / rows;
    for (int64_t e = threadIdx.x; e < E; e += blockDim.x) a.Y[t0 * R1 + e] = Yc[e];
    gram_mode_mfma(Yc, rows, int(R1), 1, part, int(R1));
  } else {
    for (int64_t e = threadIdx.x; e < E; e += blockDim.x) part[e] = double(Yc[e]);
    __syncthreads();
  }
}

// U^(1) rows of the span from the temporal pass, Y V diag(1 / s), and the
// partial Gram of those rows (r_1 x r_1).
__global__ __launch_bounds__(NT_LEAF, 2) void stream_u1_kernel(StreamArgs a, const double* V, const double* sv,
                                                                double* U64) {
  const int64_t t0 = int64_t(blockIdx.x) * a.span;
  const int64_t rows = span_rows(a, t0);
  const int r = a.rq[0];
  int64_t R1 = 1;
  for (int m = 1; m < a.p; ++m) R1 *= a.rq[m];
  for (int64_t e = threadIdx.x; e < rows * r; e += blockDim.x) {
    const int64_t t = t0 + e / r;
    const int j = int(e % r);
    const float* y = a.Y + t * R1;
    double acc = 0.0;
    for (int64_t c = 0; c < R1; ++c) acc += double(y[c]) * V[c * r + j];
    U64[t * r + j] = sv[j] > 0.0 ? acc / sv[j] : 0.0;
  }
  __syncthreads();
  double* part = a.part + int64_t(blockIdx.x) * a.part_elems;
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int i = e / r, j = e % r;
    double acc = 0.0;
    for (int64_t t = t0; t < t0 + rows; ++t) acc += U64[t * r + i] * U64[t * r + j];
    part[e] = acc;
  }
}

// U^(1) <- U^(1) R^{-1} (the Cholesky QR step), and its FP32 copy.
__global__ __launch_bounds__(NT_LEAF, 2) void stream_u1_fix_kernel(StreamArgs a, const double* Rinv, double* U64,
                                                                    float* U32) {
  const int64_t t0 = int64_t(blockIdx.x) * a.span;
  const int64_t rows = span_rows(a, t0);
  const int r = a.rq[0];
  __shared__ double row[NT_LEAF / 8][32];
  // rows in groups that fit: each group's old values are read before any is rewritten
  const int per = NT_LEAF / 8 < int(rows) ? NT_LEAF / 8 : int(rows);
  for (int64_t g = 0; g < rows; g += per) {
    const int n = rows - g < per ? int(rows - g) : per;
    for (int e = threadIdx.x; e < n * r; e += blockDim.x) row[e / r][e % r] = U64[(t0 + g + e / r) * r + e % r];
    __syncthreads();
    for (int e = threadIdx.x; e < n * r; e += blockDim.x) {
      const int i = e / r, j = e % r;
      double acc = 0.0;
      for (int k = 0; k <= j; ++k) acc += row[i][k] * Rinv[k * r + j];
      U64[(t0 + g + i) * r + j] = acc;
      U32[(t0 + g + i) * r + j] = float(acc);
    }
    __syncthreads();
  }
}

__global__ void stream_reduce_kernel(const double* part, int64_t n_parts, int64_t E, double* out64, float* out32) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < E; e += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int64_t b = 0; b < n_parts; ++b) s += part[b * E + e];
    if (out64) out64[e] = s;
    if (out32) out32[e] = float(s);
  }
}

__global__ __launch_bounds__(NT_LEAF, 1) void stream_solve_kernel(SolveArgs a) {
  extern __shared__ double lds[];
  __shared__ LeafShared sh;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* TMP = reinterpret_cast<double*>(a.ws + a.tmp_off);
  const int r = a.r;
  int64_t rows = 0;
  if (a.op == 0) {
    const int n = a.dims[0];
    double* Wm = n <= a.n_lds ? lds : reinterpret_cast<double*>(a.ws + a.eig_off);
    for (int64_t e = tid; e < int64_t(n) * n; e += nt) Wm[e] = a.gram[e];
    __syncthreads();
    const double* lam = eig_top(Wm, n, r, a.U64, r, sh.red, TMP, nullptr, Wm + int64_t(n) * n);
    for (int j = tid; j < r; j += nt) a.sv[j] = sqrt(fmax(lam[j], 0.0));
    rows = n;
  } else if (a.op == 1) {
    LeafLayout lo;
    lo.TMP = a.tmp_off;
    lo.EIG = a.eig_off;
    leading_left(a.Z, a.dims, a.p, a.mode, r, a.U64, a.vbuf, a.n_lds, lds, a.ws, lo, sh);
    rows = a.dims[a.mode];
    if (a.core) {  // the mode is the last: core[i][j] = sum_d Z[i][d] U[d][j]
      const int D = a.dims[a.mode];
      const int64_t R = prod_range(a.dims, 0, a.mode);
      double part = 0.0;
      for (int64_t e = tid; e < R * r; e += nt) {
        const int64_t i = e / r;
        const int j = int(e % r);
        double acc = 0.0;
        for (int d = 0; d < D; ++d) acc += double(a.Z[i * D + d]) * a.U64[int64_t(d) * r + j];
        a.core[e] = float(acc);
        part += acc * acc;
      }
      part = block_sum(part, sh.red);
      if (tid == 0) a.out[0] = part;
    }
  } else {
    // Cholesky G = R^T R of the r x r Gram of U^(1), then R^{-1} (upper)
    // into U64; a pivot at or below 1e-13 of the largest diagonal entry
    // (U^(1) rank-deficient: a zero singular value of the temporal problem)
    // leaves that column as it is
    if (tid == 0) {
      double* R = TMP;
      double dmax = 0.0;
      for (int i = 0; i < r; ++i) dmax = fmax(dmax, a.gram[i * r + i]);
      for (int e = 0; e < r * r; ++e) R[e] = 0.0;
      for (int j = 0; j < r; ++j) {
        double d = a.gram[j * r + j];
        for (int k = 0; k < j; ++k) d -= R[k * r + j] * R[k * r + j];
        const bool ok = d > 1e-13 * dmax;
        R[j * r + j] = ok ? sqrt(d) : 1.0;
        for (int i = j + 1; i < r; ++i) {
          double v = a.gram[j * r + i];
          for (int k = 0; k < j; ++k) v -= R[k * r + j] * R[k * r + i];
          R[j * r + i] = ok ? v / R[j * r + j] : 0.0;
        }
      }
      double* Ri = a.U64;
      for (int e = 0; e < r * r; ++e) Ri[e] = 0.0;
      for (int j = 0; j < r; ++j) {  // column j of R^{-1}: back substitution
        Ri[j * r + j] = 1.0 / R[j * r + j];
        for (int i = j - 1; i >= 0; --i) {
          double v = 0.0;
          for (int k = i + 1; k <= j; ++k) v += R[i * r + k] * Ri[k * r + j];
          Ri[i * r + j] = -v / R[i * r + i];
        }
      }
    }
    rows = 0;
  }
  __syncthreads();
  if (a.U32)
    for (int64_t e = tid; e < rows * r; e += nt) a.U32[e] = float(a.U64[e]);
}

// ------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------
hipError_t launch_stitch(const StitchArgs& a, int grid, size_t lds_bytes, int threads, hipStream_t stream) {
  if (grid <= 0 || a.n_jobs <= 0) return hipSuccess;
  if (grid > a.n_jobs || (!a.queue && grid != a.n_jobs)) return hipErrorInvalidValue;
  if (a.p < 2 || a.p > MAXP) return hipErrorInvalidValue;
  const bool few = a.p <= PM_FEW;
  switch (threads) {
    case 64: return few ? stitch_launch_64_4(a, grid, lds_bytes, stream) : stitch_launch_64_7(a, grid, lds_bytes, stream);
    case 128: return few ? stitch_launch_128_4(a, grid, lds_bytes, stream) : stitch_launch_128_7(a, grid, lds_bytes, stream);
    case 256: return few ? stitch_launch_256_4(a, grid, lds_bytes, stream) : stitch_launch_256_7(a, grid, lds_bytes, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_trim(const TrimChunk* chunks, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = n < (int64_t(1) << 20) ? n : (int64_t(1) << 20);
  hipLaunchKernelGGL(trim_gram_kernel, dim3(unsigned(grid)), dim3(NT_TRIM), 0, stream, chunks, n);
  return hipGetLastError();
}

hipError_t launch_reset_queue(int* queue, int n, hipStream_t stream) {
  if (!queue || n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, stream, queue, n);
  return hipGetLastError();
}

hipError_t launch_raw(const RawArgs& a, int n_jobs, size_t lds_bytes, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(raw_kernel, dim3(n_jobs), dim3(NT_LEAF), lds_bytes, stream, a);
  return hipGetLastError();
}

hipError_t launch_leaf(const LeafArgs& a, int n_jobs, size_t lds_bytes, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(leaf_kernel, dim3(n_jobs), dim3(NT_LEAF), lds_bytes, stream, a);
  return hipGetLastError();
}

hipError_t launch_stream_gram(const StreamArgs& a, int64_t n_spans, hipStream_t stream) {
  if (n_spans <= 0 || n_spans > (int64_t(1) << 20) || a.skip < 1 || a.skip >= a.p) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_gram_kernel, dim3(unsigned(n_spans)), dim3(NT_LEAF), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_stream_project(const StreamArgs& a, int64_t n_spans, hipStream_t stream) {
  if (n_spans <= 0 || n_spans > (int64_t(1) << 20) || a.skip < 0 || a.skip >= a.p) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_project_kernel, dim3(unsigned(n_spans)), dim3(NT_LEAF), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_stream_u1(const StreamArgs& a, int64_t n_spans, const double* V, const double* sv, double* U64,
                            hipStream_t stream) {
  if (n_spans <= 0 || n_spans > (int64_t(1) << 20)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_u1_kernel, dim3(unsigned(n_spans)), dim3(NT_LEAF), 0, stream, a, V, sv, U64);
  return hipGetLastError();
}

hipError_t launch_stream_u1_fix(const StreamArgs& a, int64_t n_spans, const double* Rinv, double* U64, float* U32,
                                hipStream_t stream) {
  if (n_spans <= 0 || n_spans > (int64_t(1) << 20) || a.rq[0] > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_u1_fix_kernel, dim3(unsigned(n_spans)), dim3(NT_LEAF), 0, stream, a, Rinv, U64, U32);
  return hipGetLastError();
}

hipError_t launch_stream_reduce(const double* part, int64_t n_parts, int64_t E, double* out64, float* out32,
                                hipStream_t stream) {
  if (E <= 0 || n_parts <= 0) return hipErrorInvalidValue;
  const int64_t blocks = (E + 255) / 256 < 4096 ? (E + 255) / 256 : 4096;
  hipLaunchKernelGGL(stream_reduce_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, part, n_parts, E, out64, out32);
  return hipGetLastError();
}

hipError_t launch_stream_solve(const SolveArgs& a, size_t lds_bytes, hipStream_t stream) {
  hipLaunchKernelGGL(stream_solve_kernel, dim3(1), dim3(NT_LEAF), lds_bytes, stream, a);
  return hipGetLastError();
}

hipError_t set_lds_limits(size_t stitch_bytes, size_t leaf_bytes) {
  hipError_t (*const fns[])(size_t) = {stitch_set_lds_64_4, stitch_set_lds_128_4, stitch_set_lds_256_4,
                                       stitch_set_lds_64_7, stitch_set_lds_128_7, stitch_set_lds_256_7};
  for (auto f : fns) {
    const hipError_t e = f(stitch_bytes);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(leaf_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(leaf_bytes));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(stream_solve_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                          int(leaf_bytes));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(raw_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(leaf_bytes));
}

int stitch_blocks_per_cu(int threads, size_t lds_bytes) {
  // the many-mode instantiation: its static LDS is the larger
  int n = 0;
  if (threads == 64) n = stitch_occupancy_64_7(lds_bytes);
  if (threads == 128) n = stitch_occupancy_128_7(lds_bytes);
  if (threads == 256) n = stitch_occupancy_256_7(lds_bytes);
  return n > 0 ? n : 1;
}

size_t stitch_static_lds() { return sizeof(StitchShared<MAXP>) + sizeof(Hit) * MAXHITS + 64; }
size_t leaf_static_lds() { return sizeof(LeafShared) + 64; }

}  // namespace tk
