// Workgroup-level building blocks for the stitch and leaf kernels.
//
// Every routine is called by all threads of a workgroup and ends with a
// barrier, so its output is visible to the whole workgroup on return.
// Tensors are C-order; a mode-n view of a tensor is (a, r, b) with a the
// product of the sizes before mode n and b the product after it.
#pragma once

#include "tk_common.hpp"

namespace tk {

constexpr int NT = 256;  // threads per workgroup (four wave64 wavefronts)
constexpr int EIG_MAXK = EIG_MAXK_HOST;  // eigenvectors one eig_top call can return

// Sum of v over the workgroup; every thread gets the result.
__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// Mode product (App. A): Y[x][i][y] (+)= sum_j A(i, j) X[x][j][y] with
// A(i, j) = A[i as + j bs], i < m, j < r; accumulation in Acc.
template <typename TX, typename TA, typename TY, typename Acc>
__device__ void mode_product_t(const TX* __restrict__ X, int64_t a, int r, int64_t b,
                               const TA* __restrict__ A, int64_t as, int64_t bs, int m,
                               TY* __restrict__ Y, bool acc) {
  const int64_t total = a * int64_t(m) * b;
  for (int64_t o = threadIdx.x; o < total; o += blockDim.x) {
    const int64_t y = o % b;
    const int64_t t = o / b;
    const int i = int(t % m);
    const int64_t x = t / m;
    const TX* xp = X + x * r * b + y;
    const TA* ap = A + i * as;
    Acc s = 0;
    for (int j = 0; j < r; ++j) s += Acc(ap[j * bs]) * Acc(xp[j * b]);
    Y[o] = acc ? TY(Acc(Y[o]) + s) : TY(s);
  }
  __syncthreads();
}

// FP32 operands with FP32 accumulation (the contractions of the ALS loop).
__device__ inline void mode_product(const float* __restrict__ X, int64_t a, int r, int64_t b,
                                    const float* __restrict__ A, int64_t as, int64_t bs, int m,
                                    float* __restrict__ Y, bool acc) {
  mode_product_t<float, float, float, float>(X, a, r, b, A, as, bs, m, Y, acc);
}

// Mode Gram G = mat_n(X) mat_n(X)^T (q x q, written as FP64 with leading
// dimension ld; symmetric) for X viewed as (a, q, b).  Acc is the
// accumulation type.
template <typename Acc>
__device__ void gram_mode(const float* __restrict__ X, int64_t a, int q, int64_t b,
                          double* __restrict__ G, int ld) {
  for (int e = threadIdx.x; e < q * q; e += blockDim.x) {
    const int i = e / q, j = e % q;
    if (j < i) continue;
    Acc s = 0;
    for (int64_t x = 0; x < a; ++x) {
      const float* pi = X + (x * q + i) * b;
      const float* pj = X + (x * q + j) * b;
      for (int64_t y = 0; y < b; ++y) s += Acc(pi[y]) * Acc(pj[y]);
    }
    G[i * ld + j] = double(s);
    G[j * ld + i] = double(s);
  }
  __syncthreads();
}

// Gram over the other side: G[c1][c2] = sum_d X[x1][d][y1] X[x2][d][y2] with
// c = x b + y, N = a b; FP64 accumulation.
__device__ void gram_other(const float* __restrict__ X, int64_t a, int D, int64_t b,
                           double* __restrict__ G, int ld) {
  const int64_t N = a * b;
  for (int64_t e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int64_t i = e / N, j = e % N;
    if (j < i) continue;
    const int64_t x1 = i / b, y1 = i % b, x2 = j / b, y2 = j % b;
    double s = 0.0;
    for (int d = 0; d < D; ++d)
      s += double(X[(x1 * D + d) * b + y1]) * double(X[(x2 * D + d) * b + y2]);
    G[i * ld + j] = s;
    G[j * ld + i] = s;
  }
  __syncthreads();
}

// Orthonormalise columns idx[0..k) of W (column c at W + c n, n rows) in
// place, in FP64.  The columns are first checked: when their Gram is within
// 1e-12 of the identity nothing more is done.  Otherwise classical
// Gram-Schmidt is applied twice, column by column; a column that vanishes
// (a zero or dependent vector) is replaced by the next unit vector e_c that
// survives, so the k columns always end orthonormal when k <= n.
// coef: >= k doubles; flag: an int in LDS.
__device__ void orthonormalize_cols(double* W, int n, int k, const int* idx, double* coef, double* red,
                                    int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (k <= 0) return;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int e = tid; e < k * k; e += nt) {
    const int i = e / k, j = e % k;
    if (j < i) continue;
    const double* a = W + int64_t(idx[i]) * n;
    const double* b = W + int64_t(idx[j]) * n;
    double d = 0.0;
    for (int r = 0; r < n; ++r) d += a[r] * b[r];
    if (fabs(d - (i == j ? 1.0 : 0.0)) > 1e-12) *flag = 1;
  }
  __syncthreads();
  if (*flag == 0) return;
  int cand = 0;
  for (int j = 0; j < k && j < n; ++j) {
    double* w = W + int64_t(idx[j]) * n;
    for (int attempt = 0; attempt <= n; ++attempt) {
      for (int pass = 0; pass < 2; ++pass) {
        // all coefficients of column j at once: groups of 8 lanes per column i < j
        for (int base = 0; base < j; base += nt / 8) {
          const int i = base + tid / 8, lane = tid % 8;
          double d = 0.0;
          if (i < j) {
            const double* a = W + int64_t(idx[i]) * n;
            for (int r = lane; r < n; r += 8) d += a[r] * w[r];
          }
          for (int o = 4; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
          if (i < j && lane == 0) coef[i] = d;
        }
        __syncthreads();
        for (int r = tid; r < n; r += nt) {
          double v = w[r];
          for (int i = 0; i < j; ++i) v -= coef[i] * W[int64_t(idx[i]) * n + r];
          w[r] = v;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int r = tid; r < n; r += nt) part += w[r] * w[r];
      const double nrm = sqrt(block_sum(part, red));
      if (nrm > 0.5) {
        for (int r = tid; r < n; r += nt) w[r] /= nrm;
        __syncthreads();
        break;
      }
      for (int r = tid; r < n; r += nt) w[r] = (r == cand) ? 1.0 : 0.0;
      ++cand;
      __syncthreads();
    }
  }
}

// Orthonormalise the k columns of E (n x k, row-major, leading dimension
// lde) in FP64, as orthonormalize_cols does (used on results held outside
// the eigensolver's buffer).  coef: >= k doubles.
__device__ void orthonormalize(double* E, int n, int k, int lde, double* coef, double* red) {
  int cand = 0;
  for (int j = 0; j < k && j < n; ++j) {
    for (int attempt = 0; attempt <= n; ++attempt) {
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = threadIdx.x; i < j; i += blockDim.x) {
          double d = 0.0;
          for (int r = 0; r < n; ++r) d += E[r * lde + i] * E[r * lde + j];
          coef[i] = d;
        }
        __syncthreads();
        for (int r = threadIdx.x; r < n; r += blockDim.x) {
          double v = E[r * lde + j];
          for (int i = 0; i < j; ++i) v -= coef[i] * E[r * lde + i];
          E[r * lde + j] = v;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int r = threadIdx.x; r < n; r += blockDim.x) part += E[r * lde + j] * E[r * lde + j];
      const double nrm = sqrt(block_sum(part, red));
      if (nrm > 0.5) {
        for (int r = threadIdx.x; r < n; r += blockDim.x) E[r * lde + j] /= nrm;
        __syncthreads();
        break;
      }
      for (int r = threadIdx.x; r < n; r += blockDim.x) E[r * lde + j] = (r == cand) ? 1.0 : 0.0;
      ++cand;
      __syncthreads();
    }
  }
  for (int j = n; j < k; ++j)
    for (int r = threadIdx.x; r < n; r += blockDim.x) E[r * lde + j] = 0.0;
  __syncthreads();
}

// Leading eigenpairs of a symmetric positive semi-definite n x n matrix S by
// one-sided Jacobi (Hestenes 1958): W (holding S, column c at W + c n) is
// rotated by plane rotations V until its columns are mutually orthogonal,
// W = S V; then V holds eigenvectors of S and column c of W equals
// lambda_c v_c.  Pairs are visited in the round-robin order, n/2 disjoint
// pairs per step, each pair by a group of g lanes of one wavefront.
// Writes the k leading unit eigenvectors into E (n x k, row-major, lde) in
// descending eigenvalue order and returns a pointer to the k eigenvalues.
// Columns whose eigenvalue is at most keep_rel times the largest are
// normalised but not orthonormalised (callers that drop such directions pass
// keep_rel > 0); with keep_rel = 0 all k columns come out orthonormal, a
// dependent one completed by a unit vector.  W must hold eig_doubles(n)
// doubles; the scratch (norms, ranks, coefficients, eigenvalues) follows the
// matrix, and the eigenvalues stay valid until W is reused.  When k > n only
// n eigenpairs exist and the extra columns of E are zero.
struct EigCounters {
  uint64_t calls = 0, sweeps = 0, jacobi_ticks = 0, tail_ticks = 0;
};

__device__ const double* eig_top(double* W, int n, int k, double* E, int lde, double* red,
                                 double keep_rel = 0.0, EigCounters* cnt = nullptr) {
  const uint64_t t_start = wall_clock64();
  __shared__ int s_idx[EIG_MAXK];
  __shared__ int s_flag;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* scratch = W + int64_t(n) * n;
  double* nrm = scratch;
  double* coef = scratch + n;
  double* lam = scratch + 2 * n;
  if (n <= 0) return lam;
  const int N = n + (n & 1);
  const int npairs = N / 2;
  int g = 64;
  while (g > 1 && npairs * g > nt) g >>= 1;
  const int groups = nt / g;
  double tr = 0.0;
  for (int i = tid; i < n; i += nt) tr += fabs(W[i * n + i]);
  tr = block_sum(tr, red);
  const double tiny = (1e-17 * tr) * (1e-17 * tr);
  const double eps = 4e-16 * double(n > 8 ? n : 8);
  int sweeps_run = 0;
  for (int sweep = 0; sweep < 40 && N > 1; ++sweep) {
    ++sweeps_run;
    int rotated = 0;
    for (int step = 0; step < N - 1; ++step) {
      for (int base = 0; base < npairs; base += groups) {
        const int pi = base + tid / g;
        const int lane = tid % g;
        int pp = n, qq = n;
        if (pi < npairs) {
          if (pi == 0) {
            pp = N - 1;
            qq = step;
          } else {
            pp = (step + pi) % (N - 1);
            qq = (step - pi + (N - 1)) % (N - 1);
          }
        }
        const bool act = pp < n && qq < n;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (act) {
          const double* wp = W + int64_t(pp) * n;
          const double* wq = W + int64_t(qq) * n;
          for (int r = lane; r < n; r += g) {
            const double x = wp[r], y = wq[r];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
        }
        for (int o = g >> 1; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          ga += __shfl_xor(ga, o, 64);
        }
        if (act) {
          const double ab = sqrt(al * be);
          if (ab > tiny && fabs(ga) > eps * ab) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double sn = c * t;
            double* wp = W + int64_t(pp) * n;
            double* wq = W + int64_t(qq) * n;
            for (int r = lane; r < n; r += g) {
              const double x = wp[r], y = wq[r];
              wp[r] = c * x - sn * y;
              wq[r] = sn * x + c * y;
            }
            rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  const uint64_t t_jac = wall_clock64();
  // column norms = |lambda|; rank them (ties by index) and keep the top k
  for (int c = tid; c < n; c += nt) {
    double s = 0.0;
    const double* w = W + int64_t(c) * n;
    for (int r = 0; r < n; ++r) s += w[r] * w[r];
    nrm[c] = sqrt(s);
  }
  __syncthreads();
  const int kk = k < n ? k : n;
  for (int c = tid; c < n; c += nt) {
    int rank = 0;
    for (int c2 = 0; c2 < n; ++c2)
      if (nrm[c2] > nrm[c] || (nrm[c2] == nrm[c] && c2 < c)) ++rank;
    if (rank < kk) s_idx[rank] = c;
  }
  __syncthreads();
  for (int j = tid; j < kk; j += nt) lam[j] = nrm[s_idx[j]];
  __syncthreads();
  // normalise the kept columns in place, then orthonormalise the leading
  // ones (those above keep_rel, or all of them)
  const double lmax = kk > 0 ? lam[0] : 0.0;
  for (int e = tid; e < n * kk; e += nt) {
    const int j = e / n, r = e % n;
    const double s = lam[j];
    double* w = W + int64_t(s_idx[j]) * n;
    w[r] = s > 0.0 ? w[r] / s : 0.0;
  }
  __syncthreads();
  int ko = kk;
  if (keep_rel > 0.0) {
    ko = 0;
    for (int j = 0; j < kk; ++j)
      if (lam[j] > keep_rel * lmax) ko = j + 1;
  }
  orthonormalize_cols(W, n, ko, s_idx, coef, red, &s_flag);
  for (int e = tid; e < n * k; e += nt) {
    const int r = e / k, j = e % k;
    E[r * lde + j] = j < kk ? W[int64_t(s_idx[j]) * n + r] : 0.0;
  }
  __syncthreads();
  if (cnt && tid == 0) {
    cnt->calls += 1;
    cnt->sweeps += uint64_t(sweeps_run);
    cnt->jacobi_ticks += t_jac - t_start;
    cnt->tail_ticks += wall_clock64() - t_jac;
  }
  return lam;
}

}  // namespace tk
