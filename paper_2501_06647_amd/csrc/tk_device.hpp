// Workgroup-level building blocks for the stitch and leaf kernels.
//
// Every routine is called by all threads of a workgroup and ends with a
// barrier, so its output is visible to the whole workgroup on return.  The
// stitch kernel runs one wavefront per job, where these barriers reduce to
// wavefront-local ordering; the leaf kernel runs four wavefronts.
// Tensors are C-order; a mode-n view of a tensor is (a, r, b) with a the
// product of the sizes before mode n and b the product after it.
#pragma once

#include "tk_common.hpp"

namespace tk {

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------

// Sum of v over the workgroup; every thread gets the result.  red: one
// double per wavefront (unused for a single-wavefront workgroup).
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (blockDim.x <= 64) return v;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// block_sum with a single barrier: buf (one double per wavefront) must not
// be written again before a later barrier has passed.
__device__ __forceinline__ double block_sum_once(double v, double* buf) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (blockDim.x <= 64) return v;
  if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) s += buf[w];
  return s;
}

// Largest v over the workgroup with its index (smallest index on ties).
// The largest of the workgroup's values, returned to every thread.
__device__ __forceinline__ double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if (blockDim.x <= 64) return v;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < int(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
  __syncthreads();
  return m;
}

__device__ __forceinline__ void block_argmax(double& v, int& idx, double* red, int* redi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (blockDim.x <= 64) return;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = v;
    redi[threadIdx.x >> 6] = idx;
  }
  __syncthreads();
  for (int w = 0; w < int(blockDim.x >> 6); ++w)
    if (red[w] > v || (red[w] == v && redi[w] < idx)) {
      v = red[w];
      idx = redi[w];
    }
  __syncthreads();
}

// 1/x for finite nonzero x: the hardware approximation refined by two
// Newton steps (quadratic convergence to FP64 rounding).
__device__ __forceinline__ double fast_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// ---------------------------------------------------------------------------
// Contractions
// ---------------------------------------------------------------------------

// Mode product (App. A): Y[x][i][y] (+)= sum_j A(i, j) X[x][j][y] with
// A(i, j) = A[i as + j bs], i < m, j < r; accumulation in Acc.  Each thread
// takes whole fibers X[x][:][y]: the fiber is loaded once into registers and
// every output of that fiber is formed from it (A is read uniformly across
// the wavefront).  Fibers longer than RMAX fall back to one output per
// thread.
template <typename TX, typename TA, typename TY, typename Acc, int RMAX>
__device__ __forceinline__ void mode_product_fiber(const TX* __restrict__ X, int64_t a, int r, int64_t b,
                                   const TA* __restrict__ A, int64_t as, int64_t bs, int m,
                                   TY* __restrict__ Y, bool acc) {
  const int64_t nf = a * b;
  for (int64_t f = threadIdx.x; f < nf; f += blockDim.x) {
    const int64_t x = f / b, y = f % b;
    const TX* xp = X + x * r * b + y;
    Acc v[RMAX];
#pragma unroll
    for (int j = 0; j < RMAX; ++j) v[j] = j < r ? Acc(xp[j * b]) : Acc(0);
    TY* yp = Y + x * int64_t(m) * b + y;
    for (int i = 0; i < m; ++i) {
      const TA* ap = A + i * as;
      Acc s = 0;
#pragma unroll
      for (int j = 0; j < RMAX; ++j)
        if (j < r) s += Acc(ap[j * bs]) * v[j];
      yp[i * b] = acc ? TY(Acc(yp[i * b]) + s) : TY(s);
    }
  }
  __syncthreads();
}

typedef float tk_f4 __attribute__((ext_vector_type(4)));

// The same product on the matrix cores, FP32 operands and accumulation: a
// GEMM with M = m outputs, K = r, and N = a b fibers f = (x, y), in 16 x 16
// output tiles (16 outputs of 16 fibers) with v_mfma_f32_16x16x4f32 over K
// in steps of 4: lane l supplies A(16 I + l % 16, 4 c + l / 16) and X at
// fiber 16 J + l % 16, index 4 c + l / 16, and holds Y rows 16 I + 4 (l /
// 16) + v of fiber 16 J + l % 16.  A wavefront takes TB fiber tiles of one
// row tile at a time and issues the loads of all of them (four K steps per
// round) before their MFMAs: the operands come from HBM or L2, so one
// memory round trip serves TB tiles.  Each tile's K steps run in order, as
// with one tile at a time.  Y must not overlap X; with acc the tile is
// added to Y.
__device__ __forceinline__ void mode_product_mfma(const float* __restrict__ X, int64_t a, int r, int64_t b,
                                                  const float* __restrict__ A, int64_t as, int64_t bs, int m,
                                                  float* __restrict__ Y, bool acc) {
  constexpr int TB = 4;
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const int64_t F = a * b;
  const int mt = (m + 15) >> 4;
  const int64_t ngr = (((F + 15) >> 4) + TB - 1) / TB;
  for (int64_t t = w; t < int64_t(mt) * ngr; t += nw) {
    const int I = int(t % mt);
    const int64_t g = t / mt;
    // out-of-range rows, fibers and indices read a valid element, masked to 0
    const int ia = I * 16 + lr;
    const float im = ia < m ? 1.f : 0.f;
    const int64_t ic = ia < m ? ia : m - 1;
    int64_t xo[TB];
    float fm[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int64_t f = (g * TB + u) * 16 + lr;
      fm[u] = f < F ? 1.f : 0.f;
      const int64_t fc = f < F ? f : F - 1;
      xo[u] = (fc / b) * r * b + fc % b;
    }
    tk_f4 c[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) c[u] = tk_f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < r; k0 += 16) {
      float av[4], bv[TB][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = k0 + 4 * q + lk;
        const float jm = j < r ? 1.f : 0.f;
        const int64_t jc = j < r ? j : r - 1;
        av[q] = A[ic * as + jc * bs] * (im * jm);
#pragma unroll
        for (int u = 0; u < TB; ++u) bv[u][q] = X[xo[u] + jc * b] * (fm[u] * jm);
      }
#pragma unroll
      for (int u = 0; u < TB; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k0 + 4 * q < r) c[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[u][q], c[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int64_t f = (g * TB + u) * 16 + lr;
      if (f < F) {
        const int64_t x = f / b, y = f % b;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = I * 16 + 4 * lk + v;
          if (i < m) {
            const int64_t o = (x * m + i) * b + y;
            Y[o] = acc ? Y[o] + c[u][v] : c[u][v];
          }
        }
      }
    }
  }
  __syncthreads();
}

typedef __bf16 tk_b8 __attribute__((ext_vector_type(8)));

// The same product with BF16 operands (rounded to nearest even from FP32)
// and FP32 accumulation, v_mfma_f32_16x16x32_bf16 over K in steps of 32:
// lane l supplies A(16 I + l % 16, 32 c + 8 (l / 16) + v) and X at fiber
// 16 J + l % 16, index 32 c + 8 (l / 16) + v, for v < 8; the output layout
// is that of mode_product_mfma.
__device__ __forceinline__ void mode_product_bf16(const float* __restrict__ X, int64_t a, int r, int64_t b,
                                                  const float* __restrict__ A, int64_t as, int64_t bs, int m,
                                                  float* __restrict__ Y, bool acc) {
  constexpr int TB = 4;  // fiber tiles per memory round, as in mode_product_mfma
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const int64_t F = a * b;
  const int mt = (m + 15) >> 4;
  const int64_t ngr = (((F + 15) >> 4) + TB - 1) / TB;
  for (int64_t t = w; t < int64_t(mt) * ngr; t += nw) {
    const int I = int(t % mt);
    const int64_t g = t / mt;
    const int ia = I * 16 + lr;
    const float im = ia < m ? 1.f : 0.f;
    const int64_t ic = ia < m ? ia : m - 1;
    int64_t xo[TB];
    float fm[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int64_t f = (g * TB + u) * 16 + lr;
      fm[u] = f < F ? 1.f : 0.f;
      const int64_t fc = f < F ? f : F - 1;
      xo[u] = (fc / b) * r * b + fc % b;
    }
    tk_f4 c[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) c[u] = tk_f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < r; k0 += 32) {
      tk_b8 av, bv[TB];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int j = k0 + 8 * lk + v;
        const float jm = j < r ? 1.f : 0.f;
        const int64_t jc = j < r ? j : r - 1;
        av[v] = (__bf16)(A[ic * as + jc * bs] * (im * jm));
#pragma unroll
        for (int u = 0; u < TB; ++u) bv[u][v] = (__bf16)(X[xo[u] + jc * b] * (fm[u] * jm));
      }
#pragma unroll
      for (int u = 0; u < TB; ++u) c[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[u], c[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int64_t f = (g * TB + u) * 16 + lr;
      if (f < F) {
        const int64_t x = f / b, y = f % b;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = I * 16 + 4 * lk + v;
          if (i < m) {
            const int64_t o = (x * m + i) * b + y;
            Y[o] = acc ? Y[o] + c[u][v] : c[u][v];
          }
        }
      }
    }
  }
  __syncthreads();
}

// FP32 operands with FP32 accumulation (the contractions of the ALS loop).
__device__ __forceinline__ void mode_product(const float* __restrict__ X, int64_t a, int r, int64_t b,
                                    const float* __restrict__ A, int64_t as, int64_t bs, int m,
                                    float* __restrict__ Y, bool acc) {
  mode_product_mfma(X, a, r, b, A, as, bs, m, Y, acc);
}

typedef double tk_d4 __attribute__((ext_vector_type(4)));

// C = A B in FP64 on the matrix cores (v_mfma_f64_16x16x4f64): 16 x 16
// output tiles per wavefront, K in steps of 4.  a(i, k) and b(k, j) return
// operands (called only in range), put(i, j, v) stores result (i, j).  Lane
// l supplies a(16 I + l % 16, 4 c + l / 16) and b(4 c + l / 16, 16 J + l % 16)
// and holds C(16 I + l / 16 + 4 v, 16 J + l % 16) for v < 4.
template <typename FA, typename FB, typename FP>
__device__ __forceinline__ void gemm_f64(int M, int N, int K, FA&& a, FB&& b, FP&& put) {
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const int mt = (M + 15) >> 4, ntl = (N + 15) >> 4;
  for (int t = w; t < mt * ntl; t += nw) {
    const int I = t % mt, J = t / mt;
    const int i = I * 16 + lr, j = J * 16 + lr;
    tk_d4 c = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 16) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * u + lk;
        av[u] = (i < M && k < K) ? double(a(i, k)) : 0.0;
        bv[u] = (j < N && k < K) ? double(b(k, j)) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (k0 + 4 * u < K) c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], c, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ri = I * 16 + lk + 4 * v;
      if (ri < M && j < N) put(ri, j, c[v]);
    }
  }
  __syncthreads();
}

// C = A B for a tall A (M x K, FP32 entries a(i, k)) and a small B (K x N,
// K <= 16, N <= 16, FP64 entries b(k, j)) on the FP64 matrix cores: B's
// fragment is loaded once, then each wavefront streams TB row tiles per
// round, their loads issued before any product or store.  Same layout and
// arithmetic order per tile as gemm_f64.
template <int TB, typename FA, typename FB, typename FP>
__device__ __forceinline__ void gemm_f64_tall(int M, int N, int K, FA&& a, FB&& b, FP&& put) {
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const int mt = (M + 15) >> 4;
  double bv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = 4 * u + lk;
    bv[u] = (lr < N && k < K) ? double(b(k, lr)) : 0.0;
  }
  for (int t0 = w; t0 < mt; t0 += TB * nw) {
    float av[TB][4];
#pragma unroll
    for (int g = 0; g < TB; ++g) {
      const int i = (t0 + g * nw) * 16 + lr;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 4 * u + lk;
        av[g][u] = (i < M && k < K) ? a(i, k) : 0.f;
      }
    }
#pragma unroll
    for (int g = 0; g < TB; ++g) {
      tk_d4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * u < K) c = __builtin_amdgcn_mfma_f64_16x16x4f64(double(av[g][u]), bv[u], c, 0, 0, 0);
      const int I = t0 + g * nw;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ri = I * 16 + lk + 4 * v;
        if (I < mt && ri < M && lr < N) put(ri, lr, c[v]);
      }
    }
  }
  __syncthreads();
}

// gemm_f64 for many row tiles (M >> N, as when a thin factor's rows stream
// from HBM): each wavefront takes TB tiles per round and issues the loads of
// all of them before any product or store, so one memory round trip serves
// TB tiles.  Same layout and arithmetic order per tile as gemm_f64.
template <int TB, typename FA, typename FB, typename FP>
__device__ __forceinline__ void gemm_f64_rows(int M, int N, int K, FA&& a, FB&& b, FP&& put) {
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const int mt = (M + 15) >> 4, ntl = (N + 15) >> 4;
  const int T = mt * ntl;
  for (int t0 = w; t0 < T; t0 += TB * nw) {
    tk_d4 c[TB];
#pragma unroll
    for (int g = 0; g < TB; ++g) c[g] = tk_d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 16) {
      double av[TB][4], bv[TB][4];
#pragma unroll
      for (int g = 0; g < TB; ++g) {
        const int t = t0 + g * nw;
        const int I = t % mt, J = t / mt;
        const int i = I * 16 + lr, j = J * 16 + lr;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + lk;
          av[g][u] = (t < T && i < M && k < K) ? double(a(i, k)) : 0.0;
          bv[g][u] = (t < T && j < N && k < K) ? double(b(k, j)) : 0.0;
        }
      }
#pragma unroll
      for (int g = 0; g < TB; ++g)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (k0 + 4 * u < K) c[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g][u], bv[g][u], c[g], 0, 0, 0);
    }
#pragma unroll
    for (int g = 0; g < TB; ++g) {
      const int t = t0 + g * nw;
      if (t >= T) break;
      const int I = t % mt, J = t / mt;
      const int j = J * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ri = I * 16 + lk + 4 * v;
        if (ri < M && j < N) put(ri, j, c[g][v]);
      }
    }
  }
  __syncthreads();
}

// Mode product in FP64 on the matrix cores: Y[x][i][y] (+)= sum_j A(i, j)
// X[x][j][y] (X FP32 or FP64, A and Y FP64), the layout of mode_product_mfma
// with v_mfma_f64_16x16x4f64 (fibers f = (x, y) as the N dimension), four
// fiber tiles per memory round as there.
template <typename TX>
__device__ __forceinline__ void mode_product_f64(const TX* __restrict__ X, int64_t a, int r, int64_t b,
                                                 const double* __restrict__ A, int64_t as, int64_t bs, int m,
                                                 double* __restrict__ Y, bool acc) {
  constexpr int TB = 4;
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const int64_t F = a * b;
  const int mt = (m + 15) >> 4;
  const int64_t ngr = (((F + 15) >> 4) + TB - 1) / TB;
  for (int64_t t = w; t < int64_t(mt) * ngr; t += nw) {
    const int I = int(t % mt);
    const int64_t g = t / mt;
    const int ia = I * 16 + lr;
    const bool iav = ia < m;
    int64_t xo[TB];
    bool fv[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int64_t f = (g * TB + u) * 16 + lr;
      fv[u] = f < F;
      xo[u] = fv[u] ? (f / b) * r * b + f % b : 0;
    }
    tk_d4 c[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) c[u] = tk_d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < r; k0 += 16) {
      double av[4], bv[TB][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = k0 + 4 * q + lk;
        av[q] = (iav && j < r) ? A[int64_t(ia) * as + int64_t(j) * bs] : 0.0;
#pragma unroll
        for (int u = 0; u < TB; ++u) bv[u][q] = (fv[u] && j < r) ? double(X[xo[u] + int64_t(j) * b]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < TB; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k0 + 4 * q < r) c[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[u][q], c[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      if (!fv[u]) continue;
      const int64_t f = (g * TB + u) * 16 + lr;
      const int64_t x = f / b, y = f % b;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = I * 16 + lk + 4 * v;
        if (i < m) {
          const int64_t o = (x * m + i) * b + y;
          Y[o] = acc ? Y[o] + c[u][v] : c[u][v];
        }
      }
    }
  }
  __syncthreads();
}

// Mode Gram on the matrix cores: G = mat_n(X) mat_n(X)^T (q x q, FP64, leading
// dimension ld; both triangles written) for X (FP32) viewed as (a, q, b).
// Each wavefront takes 16 x 16 tiles of the upper triangle and accumulates
// them with v_mfma_f64_16x16x4f64 over the a b columns, four per step: lane
// l supplies row 16 I + l % 16 (and 16 J + l % 16) of column 4 c + l / 16,
// and holds G[16 I + l / 16 + 4 v][16 J + l % 16] for v < 4.  The FP32
// products are exact in FP64 and the sums are FP64.  For q <= 48 a
// wavefront loads the column block of every row tile once per round (four
// columns) and feeds all its tiles from those registers (gram_mode_panel),
// so a round costs one memory round trip whatever the tile count; each
// tile's column steps run in the same order either way.
template <int NB>
__device__ __forceinline__ void gram_mode_panel(const float* __restrict__ X, int64_t a, int q, int64_t b,
                                                double* __restrict__ G, int ld) {
  constexpr int NT = NB * (NB + 1) / 2;
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const int64_t N = a * b;
  tk_d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = tk_d4{0.0, 0.0, 0.0, 0.0};
  int64_t x = lk / b, y = lk % b;
  const int64_t xs = 4 / b, ys = 4 % b;
  for (int64_t k0 = 0; k0 < N; k0 += 16) {
    float v[NB][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = k0 + 4 * u + lk < N;
      const float* col = X + x * q * b + y;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi) {
        const int row = bi * 16 + lr;
        v[bi][u] = (in && row < q) ? col[int64_t(row) * b] : 0.f;
      }
      x += xs;
      y += ys;
      if (y >= b) {
        y -= b;
        ++x;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (k0 + 4 * u >= N) break;
      int t = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj, ++t)
          if (t % nw == w)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(double(v[bi][u]), double(v[bj][u]), acc[t], 0, 0, 0);
    }
  }
  int t = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NB; ++bj, ++t) {
      if (t % nw != w) continue;
      const int cj = bj * 16 + lr;
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int ri = bi * 16 + lk + 4 * vv;
        if (ri < q && cj < q) {
          G[int64_t(ri) * ld + cj] = acc[t][vv];
          G[int64_t(cj) * ld + ri] = acc[t][vv];
        }
      }
    }
  __syncthreads();
}

// G = V^T V (q x q, FP64, leading dimension ld, both triangles) for a
// matrix V of D rows whose column c < q <= 16 NB is the strided FP32 vector
// p_c[d s_c], d < D (col(c, &p_c, &s_c) names it): gram_mode_panel's scheme
// with the D rows summed, each lane's column pointers fixed for the call.
// The column steps run in the order of gemm_f64 over the same operands.
template <int NB, typename FC>
__device__ __forceinline__ void gram_cols_panel(int D, int q, FC&& col, double* __restrict__ G, int ld) {
  constexpr int NT = NB * (NB + 1) / 2;
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int lr = l & 15, lk = l >> 4;
  const float* cp[NB];
  int64_t cs[NB];
#pragma unroll
  for (int bi = 0; bi < NB; ++bi) {
    const int c = bi * 16 + lr;
    cp[bi] = nullptr;
    cs[bi] = 0;
    if (c < q) col(c, &cp[bi], &cs[bi]);
  }
  tk_d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = tk_d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < D; k0 += 16) {
    float v[NB][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int d = k0 + 4 * u + lk;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi) v[bi][u] = (d < D && cp[bi]) ? cp[bi][int64_t(d) * cs[bi]] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (k0 + 4 * u >= D) break;
      int t = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj, ++t)
          if (t % nw == w)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(double(v[bi][u]), double(v[bj][u]), acc[t], 0, 0, 0);
    }
  }
  int t = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NB; ++bj, ++t) {
      if (t % nw != w) continue;
      const int cj = bj * 16 + lr;
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int ri = bi * 16 + lk + 4 * vv;
        if (ri < q && cj < q) {
          G[int64_t(ri) * ld + cj] = acc[t][vv];
          G[int64_t(cj) * ld + ri] = acc[t][vv];
        }
      }
    }
  __syncthreads();
}

__device__ __forceinline__ void gram_mode_mfma(const float* __restrict__ X, int64_t a, int q, int64_t b,
                                               double* __restrict__ G, int ld) {
  if (q <= 16) return gram_mode_panel<1>(X, a, q, b, G, ld);
  if (q <= 32) return gram_mode_panel<2>(X, a, q, b, G, ld);
  if (q <= 48) return gram_mode_panel<3>(X, a, q, b, G, ld);
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int nb = (q + 15) >> 4;
  const int ntiles = nb * (nb + 1) / 2;
  const int64_t N = a * b;
  const int lr = l & 15, lk = l >> 4;
  for (int t = w; t < ntiles; t += nw) {
    int bi = 0, rem = t;
    while (rem >= nb - bi) {
      rem -= nb - bi;
      ++bi;
    }
    const int bj = bi + rem;
    const int i = bi * 16 + lr, j = bj * 16 + lr;
    const bool iv = i < q, jv = j < q;
    const int64_t io = int64_t(i) * b, jo = int64_t(j) * b;
    tk_d4 acc = {0.0, 0.0, 0.0, 0.0};
    // this lane's column k = 4 c + lk as (x, y), advanced by 4 per step
    int64_t x = lk / b, y = lk % b;
    const int64_t xs = 4 / b, ys = 4 % b;
    // eight steps per round: the loads of a round are issued before its MFMAs
    for (int64_t k0 = 0; k0 < N; k0 += 32) {
      double av[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        av[u] = 0.0;
        bv[u] = 0.0;
        if (k0 + 4 * u + lk < N) {
          const float* col = X + x * q * b + y;
          av[u] = iv ? double(col[io]) : 0.0;
          bv[u] = jv ? double(col[jo]) : 0.0;
        }
        x += xs;
        y += ys;
        if (y >= b) {
          y -= b;
          ++x;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + 4 * u < N) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    const int cj = bj * 16 + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ri = bi * 16 + lk + 4 * v;
      if (ri < q && cj < q) {
        G[int64_t(ri) * ld + cj] = acc[v];
        G[int64_t(cj) * ld + ri] = acc[v];
      }
    }
  }
  __syncthreads();
}

// Mode Gram with BF16 operands and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16, 32 columns per step; lane l supplies rows
// 16 I + l % 16 and 16 J + l % 16 of columns 32 c + 8 (l / 16) + v), stored
// as FP64 like gram_mode_mfma.
// gram_mode_bf16 for q <= 16 NB: each round loads the 32-column block of
// every row tile once and feeds all the wavefront's tiles of the upper
// triangle from those registers (same per-tile arithmetic).
template <int NB>
__device__ __forceinline__ void gram_mode_bf16_panel(const float* __restrict__ X, int64_t a, int q, int64_t b,
                                                     double* __restrict__ G, int ld) {
  constexpr int NT = NB * (NB + 1) / 2;
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int64_t N = a * b;
  const int lr = l & 15, lk = l >> 4;
  int64_t ro[NB];
  float rm[NB];
#pragma unroll
  for (int bi = 0; bi < NB; ++bi) {
    const int i = bi * 16 + lr;
    rm[bi] = i < q ? 1.f : 0.f;
    ro[bi] = int64_t(i < q ? i : q - 1) * b;
  }
  tk_f4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = tk_f4{0.f, 0.f, 0.f, 0.f};
  int64_t x = (8 * lk) / b, y = (8 * lk) % b;
  const int64_t xs = 32 / b, ys = 32 % b;
  for (int64_t k0 = 0; k0 < N; k0 += 32) {
    tk_b8 v[NB];
    int64_t xv = x, yv = y;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const bool kin = k0 + 8 * lk + e < N;
      const float* col = X + (kin ? xv * q * b + yv : 0);
      const float km = kin ? 1.f : 0.f;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi) v[bi][e] = (__bf16)(col[ro[bi]] * (rm[bi] * km));
      if (++yv == b) {
        yv = 0;
        ++xv;
      }
    }
    int t = 0;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
      for (int bj = bi; bj < NB; ++bj, ++t)
        if (t % nw == w) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(v[bi], v[bj], acc[t], 0, 0, 0);
    x += xs;
    y += ys;
    if (y >= b) {
      y -= b;
      ++x;
    }
  }
  int t = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NB; ++bj, ++t) {
      if (t % nw != w) continue;
      const int cj = bj * 16 + lr;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ri = bi * 16 + 4 * lk + e;
        if (ri < q && cj < q) {
          G[int64_t(ri) * ld + cj] = double(acc[t][e]);
          G[int64_t(cj) * ld + ri] = double(acc[t][e]);
        }
      }
    }
  __syncthreads();
}

__device__ __forceinline__ void gram_mode_bf16(const float* __restrict__ X, int64_t a, int q, int64_t b,
                                               double* __restrict__ G, int ld) {
  if (q <= 16) return gram_mode_bf16_panel<1>(X, a, q, b, G, ld);
  if (q <= 32) return gram_mode_bf16_panel<2>(X, a, q, b, G, ld);
  if (q <= 48) return gram_mode_bf16_panel<3>(X, a, q, b, G, ld);
  const int nw = int(blockDim.x) >> 6, w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const int nb = (q + 15) >> 4;
  const int ntiles = nb * (nb + 1) / 2;
  const int64_t N = a * b;
  const int lr = l & 15, lk = l >> 4;
  for (int t = w; t < ntiles; t += nw) {
    int bi = 0, rem = t;
    while (rem >= nb - bi) {
      rem -= nb - bi;
      ++bi;
    }
    const int bj = bi + rem;
    const int i = bi * 16 + lr, j = bj * 16 + lr;
    const float imk = i < q ? 1.f : 0.f, jmk = j < q ? 1.f : 0.f;
    const int64_t io = int64_t(i < q ? i : q - 1) * b, jo = int64_t(j < q ? j : q - 1) * b;
    tk_f4 acc = {0.f, 0.f, 0.f, 0.f};
    // this lane's first column 32 c + 8 lk as (x, y), advanced by 32 per step
    int64_t x = (8 * lk) / b, y = (8 * lk) % b;
    const int64_t xs = 32 / b, ys = 32 % b;
    for (int64_t k0 = 0; k0 < N; k0 += 32) {
      tk_b8 av, bv;
      int64_t xv = x, yv = y;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const bool kin = k0 + 8 * lk + v < N;
        const float* col = X + (kin ? xv * q * b + yv : 0);
        const float km = kin ? 1.f : 0.f;
        av[v] = (__bf16)(col[io] * (imk * km));
        bv[v] = (__bf16)(col[jo] * (jmk * km));
        if (++yv == b) {
          yv = 0;
          ++xv;
        }
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
      x += xs;
      y += ys;
      if (y >= b) {
        y -= b;
        ++x;
      }
    }
    const int cj = bj * 16 + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ri = bi * 16 + 4 * lk + v;
      if (ri < q && cj < q) {
        G[int64_t(ri) * ld + cj] = double(acc[v]);
        G[int64_t(cj) * ld + ri] = double(acc[v]);
      }
    }
  }
  __syncthreads();
}

// Gram of the rows of a tall, narrow matrix: G = V^T V for V (l x k,
// row-major), FP64 accumulation, k <= 32.  Threads split the rows; each owns
// a 4 x 4 tile of G for its share of rows, and the partial tiles are summed
// through part (ntiles x nsplit x 16 doubles, at most max_parts x 16, for
// any workgroup size).
__device__ __forceinline__ void gram_rows(const float* __restrict__ V, int64_t l, int k, double* __restrict__ G,
                                          int ld, double* __restrict__ part, int max_parts = GRAM_ROWS_TILES) {
  const int nb = (k + 3) / 4;
  const int ntiles = nb * (nb + 1) / 2;
  const int nsplit = gram_rows_split(ntiles, int(blockDim.x), max_parts);
  for (int w = threadIdx.x; w < ntiles * nsplit; w += blockDim.x) {
    const int t = w % ntiles, sp = w / ntiles;
    int bi = 0, rem = t;
    while (rem >= nb - bi) {
      rem -= nb - bi;
      ++bi;
    }
    const int bj = bi + rem;
    double s[4][4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) s[ii][jj] = 0.0;
    // four rows per round, all their loads issued before the products, so
    // that one memory round trip serves four rows (the rows stream from
    // HBM); the sums keep the row order
    int64_t r = sp;
    for (; r + 3 * int64_t(nsplit) < l; r += 4 * int64_t(nsplit)) {
      float u[4][4], v[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float* row = V + (r + q * int64_t(nsplit)) * k;
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          u[q][ii] = bi * 4 + ii < k ? row[bi * 4 + ii] : 0.0f;
          v[q][ii] = bj * 4 + ii < k ? row[bj * 4 + ii] : 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) s[ii][jj] += double(u[q][ii]) * double(v[q][jj]);
    }
    for (; r < l; r += nsplit) {
      const float* row = V + r * k;
      double u[4], v[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        u[ii] = bi * 4 + ii < k ? double(row[bi * 4 + ii]) : 0.0;
        v[ii] = bj * 4 + ii < k ? double(row[bj * 4 + ii]) : 0.0;
      }
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) s[ii][jj] += u[ii] * v[jj];
    }
    double* pp = part + (int64_t(t) * nsplit + sp) * 16;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) pp[ii * 4 + jj] = s[ii][jj];
  }
  __syncthreads();
  for (int w = threadIdx.x; w < ntiles * 16; w += blockDim.x) {
    const int t = w / 16, e = w % 16;
    int bi = 0, rem = t;
    while (rem >= nb - bi) {
      rem -= nb - bi;
      ++bi;
    }
    const int bj = bi + rem;
    double acc = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) acc += part[(int64_t(t) * nsplit + sp) * 16 + e];
    const int i = bi * 4 + e / 4, j = bj * 4 + e % 4;
    if (i < k && j < k) {
      G[i * ld + j] = acc;
      G[j * ld + i] = acc;
    }
  }
  __syncthreads();
}

// Gram over the other side: G[c1][c2] = sum_d X[x1][d][y1] X[x2][d][y2] with
// c = x b + y, N = a b; FP64 accumulation.
__device__ __forceinline__ void gram_other(const float* __restrict__ X, int64_t a, int D, int64_t b,
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

// ---------------------------------------------------------------------------
// Orthonormalisation
// ---------------------------------------------------------------------------

// Orthonormalise the k columns of E (n rows; entry (r, j) at E[r rs + j cs];
// FP64) in place: if their Gram is within 1e-12 of the identity nothing
// changes; otherwise classical Gram-Schmidt is applied twice, column by
// column, and a column that vanishes (a zero or dependent vector) is replaced
// by the next unit vector that survives, so the k columns end orthonormal
// when k <= n (columns beyond n are zeroed).  coef: >= k doubles; flag: an
// int in LDS.
__device__ __forceinline__ void orthonormalize(double* E, int n, int k, int64_t rs, int64_t cs, double* coef, double* red,
                               int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (k <= 0) return;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int e = tid; e < k * k; e += nt) {
    const int i = e / k, j = e % k;
    if (j < i) continue;
    double d = 0.0;
    for (int r = 0; r < n; ++r) d += E[r * rs + i * cs] * E[r * rs + j * cs];
    if (fabs(d - (i == j ? 1.0 : 0.0)) > 1e-12) *flag = 1;
  }
  __syncthreads();
  if (*flag == 0) return;
  int cand = 0;
  for (int j = 0; j < k && j < n; ++j) {
    for (int attempt = 0; attempt <= n; ++attempt) {
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = tid; i < j; i += nt) {
          double d = 0.0;
          for (int r = 0; r < n; ++r) d += E[r * rs + i * cs] * E[r * rs + j * cs];
          coef[i] = d;
        }
        __syncthreads();
        for (int r = tid; r < n; r += nt) {
          double v = E[r * rs + j * cs];
          for (int i = 0; i < j; ++i) v -= coef[i] * E[r * rs + i * cs];
          E[r * rs + j * cs] = v;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int r = tid; r < n; r += nt) part += E[r * rs + j * cs] * E[r * rs + j * cs];
      const double nrm = sqrt(block_sum(part, red));
      if (nrm > 0.5) {
        for (int r = tid; r < n; r += nt) E[r * rs + j * cs] /= nrm;
        __syncthreads();
        break;
      }
      for (int r = tid; r < n; r += nt) E[r * rs + j * cs] = (r == cand) ? 1.0 : 0.0;
      ++cand;
      __syncthreads();
    }
  }
  for (int j = n; j < k; ++j)
    for (int r = tid; r < n; r += nt) E[r * rs + j * cs] = 0.0;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Pivoted Cholesky
// ---------------------------------------------------------------------------

// Pivoted Cholesky in place (right-looking, symmetric pivoting by swapping
// rows and columns; Golub & Van Loan's outer-product form): G (m x m,
// row-major, symmetric, both triangles valid) is overwritten so that its
// lower triangle holds L with P^T G P = L L^T (row and column i belong to
// pivot position i; piv[i] is the original index), the pivot being the
// largest remaining diagonal; it stops when that diagonal is at most tau
// times the largest initial one and returns that rank q (columns >= q of L
// are not a factor).  Every step touches only the trailing block, four
// entries per round with their loads issued first, so the factorisation
// stays wherever G is (LDS for the sizes that matter).
__device__ __forceinline__ int pchol_inplace(double* G, int m, double tau, int* piv, double* red, int* redi) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double dmax0 = 0.0;
  for (int i = tid; i < m; i += nt) {
    piv[i] = i;
    dmax0 = fmax(dmax0, G[int64_t(i) * m + i]);
  }
  int dummy = 0;
  block_argmax(dmax0, dummy, red, redi);
  __syncthreads();
  int q = m;
  for (int j = 0; j < m; ++j) {
    double bv = -1.0;
    int bi = m;
    for (int i = j + tid; i < m; i += nt) {
      const double v = G[int64_t(i) * m + i];
      if (v > bv || (v == bv && i < bi)) {
        bv = v;
        bi = i;
      }
    }
    block_argmax(bv, bi, red, redi);
    if (!(bv > tau * dmax0) || !(bv > 0.0)) {
      q = j;
      break;
    }
    if (bi != j) {  // rows j and bi (every column), then columns j and bi (every row)
      for (int c = tid; c < m; c += nt) {
        const double x = G[int64_t(j) * m + c];
        G[int64_t(j) * m + c] = G[int64_t(bi) * m + c];
        G[int64_t(bi) * m + c] = x;
      }
      __syncthreads();
      for (int r = tid; r < m; r += nt) {
        const double x = G[int64_t(r) * m + j];
        G[int64_t(r) * m + j] = G[int64_t(r) * m + bi];
        G[int64_t(r) * m + bi] = x;
      }
      if (tid == 0) {
        const int x = piv[j];
        piv[j] = piv[bi];
        piv[bi] = x;
      }
      __syncthreads();
    }
    const double ljj = sqrt(bv);
    const double inv = 1.0 / ljj;
    for (int i = j + 1 + tid; i < m; i += nt) {
      const double l = G[int64_t(i) * m + j] * inv;
      G[int64_t(i) * m + j] = l;
      G[int64_t(j) * m + i] = l;
    }
    if (tid == 0) G[int64_t(j) * m + j] = ljj;
    __syncthreads();
    // trailing update G[i][k] -= L[i][j] L[k][j] over the whole block (it stays symmetric)
    const int mm = m - j - 1;
    const int tot = mm * mm;
    int e = tid;
    for (; e + 3 * nt < tot; e += 4 * nt) {
      int ii[4], kk[4];
      double g[4], li[4], lk[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int eu = e + u * nt;
        ii[u] = j + 1 + eu / mm;
        kk[u] = j + 1 + eu % mm;
        g[u] = G[int64_t(ii[u]) * m + kk[u]];
        li[u] = G[int64_t(ii[u]) * m + j];
        lk[u] = G[int64_t(kk[u]) * m + j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) G[int64_t(ii[u]) * m + kk[u]] = g[u] - li[u] * lk[u];
    }
    for (; e < tot; e += nt) {
      const int i = j + 1 + e / mm, k = j + 1 + e % mm;
      G[int64_t(i) * m + k] -= G[int64_t(i) * m + j] * G[int64_t(k) * m + j];
    }
    __syncthreads();
  }
  __syncthreads();
  return q;
}

// From pchol_inplace's result (L in the lower triangle of G, piv, rank q)
// for the Gram V^T V of a matrix V with m columns: the coordinates C (q x m,
// leading dimension ldc) of V's columns in the orthonormal basis
// B = V P [L11^{-T}; 0], C = B^T V = L^T P^T, then F (m x q, leading
// dimension ldf) with B = V F.  L11^{-1} overwrites L11 in place, column by
// column from the last (each a triangular product with the columns already
// inverted, rows in parallel); col: m doubles of scratch.
template <typename TC>
__device__ __forceinline__ void pchol_basis_inplace(double* G, const int* piv, int m, int q, TC* C, int ldc, double* F,
                                                    int ldf, double* col) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < q * m; e += nt) {
    const int j = e / m, c = e % m;
    C[int64_t(j) * ldc + piv[c]] = TC(c >= j ? G[int64_t(c) * m + j] : 0.0);
  }
  __syncthreads();
  for (int j = q - 1; j >= 0; --j) {
    for (int i = j + tid; i < q; i += nt) col[i] = G[int64_t(i) * m + j];
    __syncthreads();
    const double djj = 1.0 / col[j];
    for (int i = j + 1 + tid; i < q; i += nt) {
      // T[i][j] = -T[j][j] sum_{t=j+1..i} T[i][t] L[t][j]  (columns > j already hold T)
      const double* Ti = G + int64_t(i) * m;
      double acc = 0.0;
      int t = j + 1;
      for (; t + 3 <= i; t += 4) {
        const double a0 = Ti[t], a1 = Ti[t + 1], a2 = Ti[t + 2], a3 = Ti[t + 3];
        acc += a0 * col[t];
        acc += a1 * col[t + 1];
        acc += a2 * col[t + 2];
        acc += a3 * col[t + 3];
      }
      for (; t <= i; ++t) acc += Ti[t] * col[t];
      G[int64_t(i) * m + j] = -djj * acc;
    }
    if (tid == 0) G[int64_t(j) * m + j] = djj;
    __syncthreads();
  }
  for (int e = tid; e < m * q; e += nt) {
    const int c = e / q, j = e % q;
    F[int64_t(piv[c]) * ldf + j] = (c < q && j >= c) ? G[int64_t(j) * m + c] : 0.0;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Symmetric eigenproblems
// ---------------------------------------------------------------------------

struct EigCounters {  // zeroed by the owner (it may live in LDS)
  uint64_t calls, sweeps, values_ticks, tail_ticks, fallbacks;
  uint64_t tri_ticks, invit_ticks;  // parts of the two above: tridiagonalisation, inverse iteration
  uint64_t warm, warm_fail, warm_steps, warm_ticks;  // eig_top_warm: accepted, refused, steps, time
  uint64_t warm_rr_ticks;                            // the part of warm_ticks in Rayleigh-Ritz
};

// Leading eigenpairs of a symmetric n x n matrix S through the tridiagonal
// route (Golub & Van Loan, Secs. 8.3-8.4; the scheme of LAPACK's
// dsytrd/dstebz/dstein/dormtr):
//   1. Householder tridiagonalisation Q^T S Q = T (S in W is overwritten;
//      reflector i is kept in column i of W below the subdiagonal);
//   2. the k largest eigenvalues of T by multisection on Sturm counts (the
//      LDL^T pivots of T - x I), nt / k lanes per eigenvalue;
//   3. their eigenvectors by inverse iteration on T (tridiagonal LU with
//      partial pivoting, recomputed with the forward pass of each of three
//      solves, one lane per vector); vectors whose eigenvalues lie within
//      1e-9 |T| of each other are re-orthogonalised after every solve;
//   4. back-transformation by the reflectors, Rayleigh quotients for the
//      eigenvalues, and a final orthonormality check (CGS2 if needed).
// The eigenvectors live in W's free upper triangle while k < n / 2 (vector
// j in rows j and n-2-j), else in tmp.  Writes the k leading unit
// eigenvectors into E (n x k, row stride lde) in descending eigenvalue order
// (when k > n the extra columns are zero) and returns the k eigenvalues.
// W holds the n x n matrix, vec the
// eig_vec_doubles(n) doubles of vectors and workgroup partials (W + n n when
// both share one buffer); tmp: 4 n k doubles.  The returned eigenvalues
// live in vec.
__device__ __forceinline__ const double* eig_top_tri(double* W, int n, int k, double* E, int lde, double* red,
                                                     double* tmp, EigCounters* cnt, double* vec,
                                                     double* lfree = nullptr, int64_t nfree = 0) {
  __shared__ int s_flag;
  __shared__ int s_busy;
  const uint64_t t_start = wall_clock64();
  const int tid = threadIdx.x, nt = blockDim.x;
  double* d = vec;
  double* e = d + n;
  double* tau = e + n;
  double* lam = tau + n;
  double* vv = lam + n;         // reflector of the current step, then e^2
  double* pw = vv + n;          // p, then w, of the current step
  double* iv = pw + n;          // bisection brackets, two per eigenvalue
  double* part = iv + 2 * n;    // nt doubles of partial results
  if (n <= 0) return lam;
  const int kk = k < n ? k : n;

  // ---- 1. tridiagonalisation ---------------------------------------------------
  // Step i forms reflector u_i from row i, which is up to date, then makes one
  // pass over the trailing block [i+1:, i+1:] that applies the rank-two update
  // of step i-1 and accumulates p = t A u_i from the updated entries; with
  // w = p - (t/2)(p.u) u it brings row i+1 up to date right away, so the next
  // reflector is ready and the update of step i waits for the next pass.
  // Reflector/update vectors alternate between (vv, pw) and (lam, iv).
  double* red2 = red + 4;  // second reduction buffer (nt <= 256)
  double s2 = 0.0;
  if (n > 2) {
    for (int c = 2 + tid; c < n; c += nt) s2 += W[c] * W[c];
    s2 = block_sum(s2, red);
  }
  for (int i = 0; i + 2 < n; ++i) {
    const int m = n - i - 1;
    const double* Wi = W + int64_t(i) * n;  // row i
    double* uc = (i & 1) ? lam : vv;        // u_i
    double* wc = (i & 1) ? iv : pw;         // p_i, then w_i
    const double* uo = (i & 1) ? vv : lam;  // u_{i-1}
    const double* wo = (i & 1) ? pw : iv;   // w_{i-1}
    const double alpha = Wi[i + 1];
    double beta = alpha, t = 0.0, scale = 0.0;
    if (s2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      t = (beta - alpha) * fast_rcp(beta);
      scale = fast_rcp(alpha - beta);
    }
    for (int c = i + 1 + tid; c < n; c += nt) {
      const double u = c == i + 1 ? 1.0 : Wi[c] * scale;
      uc[c] = u;
      if (c > i + 1) W[int64_t(c) * n + i] = u;  // reflector -> column i
    }
    if (tid == 0) {
      d[i] = Wi[i];
      e[i] = beta;
      tau[i] = t;
    }
    __syncthreads();
    // the pass: A <- A - (u_{i-1} w_{i-1}^T + w_{i-1} u_{i-1}^T), p = t A u_i,
    // thread (r, sp) taking column r (row r by symmetry), rows c = sp mod nsplit
    const int nsplit = nt >= 2 * m ? nt / m : 1;
    const int r0 = nsplit == 1 ? tid : tid % m;
    const int sp = nsplit == 1 ? 0 : tid / m;
    const int rstep = nsplit == 1 ? nt : m;
    if (sp < nsplit) {
      for (int r = i + 1 + r0; r < n; r += rstep) {
        double acc = 0.0;
        if (i > 0) {
          const double ur = uo[r], wr = wo[r];
          int c = i + 1 + sp;
          // four entries per round: every load of the round is issued before
          // its stores, so one memory round trip serves four entries
          for (; c + 3 * nsplit < n; c += 4 * nsplit) {
            double* a0 = W + int64_t(c) * n + r;
            double* a1 = a0 + int64_t(nsplit) * n;
            double* a2 = a1 + int64_t(nsplit) * n;
            double* a3 = a2 + int64_t(nsplit) * n;
            const double y0 = *a0, y1 = *a1, y2 = *a2, y3 = *a3;
            const double p0 = uo[c], p1 = uo[c + nsplit], p2 = uo[c + 2 * nsplit], p3 = uo[c + 3 * nsplit];
            const double q0 = wo[c], q1 = wo[c + nsplit], q2 = wo[c + 2 * nsplit], q3 = wo[c + 3 * nsplit];
            const double v0 = uc[c], v1 = uc[c + nsplit], v2 = uc[c + 2 * nsplit], v3 = uc[c + 3 * nsplit];
            const double x0 = y0 - (p0 * wr + q0 * ur);
            const double x1 = y1 - (p1 * wr + q1 * ur);
            const double x2 = y2 - (p2 * wr + q2 * ur);
            const double x3 = y3 - (p3 * wr + q3 * ur);
            *a0 = x0;
            *a1 = x1;
            *a2 = x2;
            *a3 = x3;
            acc += x0 * v0;
            acc += x1 * v1;
            acc += x2 * v2;
            acc += x3 * v3;
          }
          for (; c < n; c += nsplit) {
            double* a = W + int64_t(c) * n + r;
            const double x = *a - (uo[c] * wr + wo[c] * ur);
            *a = x;
            acc += x * uc[c];
          }
        } else {
          for (int c = i + 1 + sp; c < n; c += nsplit) acc += W[int64_t(c) * n + r] * uc[c];
        }
        if (nsplit == 1)
          wc[r] = t * acc;
        else
          part[sp * m + (r - i - 1)] = acc;
      }
    }
    __syncthreads();
    // p_{i+1} for every thread (read before anyone overwrites it with w)
    double p1;
    if (nsplit == 1) {
      p1 = wc[i + 1];
    } else {
      double acc = 0.0;
      for (int q = 0; q < nsplit; ++q) acc += part[q * m];
      p1 = t * acc;
    }
    double kd = 0.0;
    for (int r = i + 1 + tid; r < n; r += nt) {
      if (nsplit > 1) {
        double acc = 0.0;
        for (int q = 0; q < nsplit; ++q) acc += part[q * m + r - i - 1];
        wc[r] = t * acc;
      }
      kd += wc[r] * uc[r];
    }
    const double K = 0.5 * t * block_sum_once(kd, red);
    const double w1 = p1 - K * uc[i + 1];
    double s2n = 0.0;
    for (int r = i + 1 + tid; r < n; r += nt) {
      const double w = wc[r] - K * uc[r];
      wc[r] = w;
      double* a = W + int64_t(i + 1) * n + r;  // row i+1 brought up to date
      const double x = *a - (uc[i + 1] * w + w1 * uc[r]);
      *a = x;
      if (r > i + 2) s2n += x * x;
    }
    s2 = block_sum_once(s2n, red2);
    if (nt <= 64) __syncthreads();  // row i+1 written before the next step reads it
  }
  __syncthreads();
  if (tid == 0) {
    if (n > 2) {  // the last step's update on the final diagonal entry
      const double* ul = ((n - 3) & 1) ? lam : vv;
      const double* wl = ((n - 3) & 1) ? iv : pw;
      W[int64_t(n - 1) * n + n - 1] -= ul[n - 1] * wl[n - 1] + wl[n - 1] * ul[n - 1];
    }
    if (n >= 2) {
      d[n - 2] = W[int64_t(n - 2) * n + n - 2];
      e[n - 2] = W[int64_t(n - 2) * n + n - 1];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = W[int64_t(n - 1) * n + n - 1];
    e[n - 1] = 0.0;
    tau[n - 1] = 0.0;
  }
  __syncthreads();

  // ---- 2. eigenvalues: multisection on Sturm counts -------------------------------
  const uint64_t t_tri = wall_clock64();
  double gmax = 0.0;
  for (int i = tid; i < n; i += nt)
    gmax = fmax(gmax, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + fabs(e[i]));
  {
    int dummy = 0;
    block_argmax(gmax, dummy, red, reinterpret_cast<int*>(part));
  }
  __syncthreads();
  if (!(gmax > 0.0)) {  // T = 0: any orthonormal basis
    for (int64_t x = tid; x < int64_t(n) * k; x += nt) {
      const int r = int(x / k), j = int(x % k);
      E[int64_t(r) * lde + j] = (j < kk && r == j) ? 1.0 : 0.0;
    }
    for (int j = tid; j < kk; j += nt) lam[j] = 0.0;
    __syncthreads();
    return lam;
  }
  const double ginv = 1.0 / gmax;
  for (int i = tid; i < n; i += nt) {
    d[i] *= ginv;
    e[i] *= ginv;
    vv[i] = e[i] * e[i];
  }
  const double pivmin = 1e-250;
  const int g = nt / kk;                // lanes per eigenvalue
  const int pl = nt <= 128 ? 2 : 1;     // points per lane (two independent Sturm chains)
  const int gp = g * pl;                // points per eigenvalue and step
  const double igp = 1.0 / double(gp + 1);
  for (int j = tid; j < kk; j += nt) {
    iv[2 * j] = -1.0 - 1e-12;
    iv[2 * j + 1] = 1.0 + 1e-12;
  }
  __syncthreads();
  int iters = 0;
  for (; iters < 80; ++iters) {
    const int j = tid / g, tg = tid % g;
    int c0 = 0, c1 = 0;
    if (j < kk) {
      const double a = iv[2 * j], b = iv[2 * j + 1];
      const double x0 = a + (b - a) * (double(pl * tg + 1) * igp);
      const double x1 = a + (b - a) * (double(pl * tg + 2) * igp);
      double q0 = d[0] - x0, q1 = d[0] - x1;
      if (fabs(q0) < pivmin) q0 = -pivmin;
      if (fabs(q1) < pivmin) q1 = -pivmin;
      c0 = q0 < 0.0 ? 1 : 0;
      c1 = q1 < 0.0 ? 1 : 0;
      for (int r = 1; r < n; ++r) {
        double y0 = __builtin_amdgcn_rcp(q0), y1 = __builtin_amdgcn_rcp(q1);
        y0 = fma(y0, fma(-q0, y0, 1.0), y0);
        y1 = fma(y1, fma(-q1, y1, 1.0), y1);
        q0 = (d[r] - x0) - vv[r - 1] * y0;
        q1 = (d[r] - x1) - vv[r - 1] * y1;
        if (fabs(q0) < pivmin) q0 = -pivmin;
        if (fabs(q1) < pivmin) q1 = -pivmin;
        c0 += q0 < 0.0 ? 1 : 0;
        c1 += q1 < 0.0 ? 1 : 0;
      }
    }
    part[pl * tid] = double(c0);
    if (pl == 2) part[pl * tid + 1] = double(c1);
    __syncthreads();
    int open = 0;
    if (j < kk && tg == 0) {
      const int idx = n - 1 - j;  // ascending index of the eigenvalue
      const double a = iv[2 * j], b = iv[2 * j + 1];
      double na = a, nb = b;
      for (int u = 0; u < gp; ++u) {
        const double xu = a + (b - a) * (double(u + 1) * igp);
        if (int(part[j * gp + u]) <= idx) na = xu;
        else if (nb == b) nb = xu;
      }
      iv[2 * j] = na;
      iv[2 * j + 1] = nb;
      open = (nb - na) > 1e-13 * fmax(1.0, fabs(na) + fabs(nb)) ? 1 : 0;
    }
    if (!__syncthreads_or(open)) break;
  }
  const uint64_t t_bis = wall_clock64();

  // ---- 3. inverse iteration on T ------------------------------------------------------
  // vector j, entry r: in W's upper triangle (rows j and n-2-j) or in tmp
  // eigenvector j, entry r: in W's free upper triangle (rows j and n-2-j)
  // while 2 k < n, else in tmp.  The two placements are separate
  // instantiations so that every access has one address space.
  struct XinW {
    double* W;
    int n;
    __device__ __forceinline__ double& operator()(int j, int r) const {
      return r < n - 1 - j ? W[int64_t(j) * n + j + 1 + r] : W[int64_t(n - 2 - j) * n + r];
    }
  };
  struct XinT {
    double* T;
    int kk;
    __device__ __forceinline__ double& operator()(int j, int r) const { return T[int64_t(r) * kk + j]; }
  };
  // pivot rows of the LU factors (n x kk each), and the vectors when they
  // do not fit in W's free triangle: in LDS when the caller has room there
  // (lfree, nfree doubles), else in tmp.  Each solve is a serial chain per
  // lane through these rows, so their latency counts in full.
  const bool lu_lds = lfree && int64_t(4) * n * kk <= nfree;
  double* U1 = lu_lds ? lfree : tmp;
  double* U2 = U1 + int64_t(n) * kk;
  double* U3 = U2 + int64_t(n) * kk;
  const double ptiny = 1e-15;  // pivot floor of the scaled problem
  int* clus = reinterpret_cast<int*>(part);  // cluster start of each eigenvalue, and its position
  if (tid == 0) {
    int maxpos = 0, start = 0;
    for (int j = 0; j < kk; ++j) {
      const double xj = 0.5 * (iv[2 * j] + iv[2 * j + 1]);
      if (j > 0 && fabs(0.5 * (iv[2 * j - 2] + iv[2 * j - 1]) - xj) > 1e-9) start = j;
      clus[2 * j] = start;
      clus[2 * j + 1] = j - start;
      if (j - start > maxpos) maxpos = j - start;
    }
    s_busy = maxpos;
  }
  uint64_t t_inv = 0;
  auto vectors = [&](auto X) {
  if (tid < kk) {  // start vector: a fixed pseudo-random pattern per eigenvalue
    for (int r = 0; r < n; ++r) {
      const uint32_t h = (uint32_t(r) * 2654435761u) ^ (uint32_t(tid + 1) * 2246822519u);
      X(tid, r) = 0.5 + double((h >> 8) & 0xFFFF) / 65536.0;
    }
  }
  __syncthreads();
  const int maxpos = s_busy;
  // a solve's output is normalised lazily: its norm is summed during the
  // back substitution and the scale sc applied when the next solve reads
  // the right-hand side (or by an explicit pass after the last solve)
  double sc = 1.0;
  for (int it = 0; it < 3; ++it) {
    if (tid < kk) {
      const int j = tid;
      const double sg = 0.5 * (iv[2 * j] + iv[2 * j + 1]);
      // LU of T - sg I with partial pivoting, applied to the right-hand side
      // as it is formed; U rows stored for the back substitution
      double w0 = d[0] - sg, w1 = n > 1 ? e[0] : 0.0;
      double xr = X(j, 0) * sc;
      for (int r = 0; r + 1 < n; ++r) {
        const double c = e[r], a1 = d[r + 1] - sg, b1 = r + 2 < n ? e[r + 1] : 0.0;
        const double xs = X(j, r + 1) * sc;
        const int64_t o = int64_t(r) * kk + j;
        double nxr;
        if (fabs(w0) >= fabs(c)) {
          if (fabs(w0) < ptiny) w0 = w0 < 0.0 ? -ptiny : ptiny;
          const double inv = fast_rcp(w0);
          const double l = c * inv;
          U1[o] = inv;  // reciprocal pivot
          U2[o] = w1;
          U3[o] = 0.0;
          X(j, r) = xr;
          nxr = xs - l * xr;
          w0 = a1 - l * w1;
          w1 = b1;
        } else {
          const double inv = fast_rcp(c);
          const double l = w0 * inv;
          U1[o] = inv;
          U2[o] = a1;
          U3[o] = b1;
          X(j, r) = xs;
          nxr = xr - l * xs;
          w0 = w1 - l * a1;
          w1 = -l * b1;
        }
        xr = nxr;
      }
      if (fabs(w0) < ptiny) w0 = w0 < 0.0 ? -ptiny : ptiny;
      // back substitution, eight rows per round with their factors loaded
      // first; values carried in registers.  Should a component exceed
      // 1e150 the whole system (solved part and remaining right-hand side)
      // is scaled by 1e-150.
      double x1 = xr / w0, x2 = 0.0;
      X(j, n - 1) = x1;
      double ss = x1 * x1;
      for (int r0 = n - 2; r0 >= 0; r0 -= 8) {
        double u1[8], u2[8], u3[8], rh[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = r0 - u;
          if (r >= 0) {
            const int64_t o = int64_t(r) * kk + j;
            u1[u] = U1[o];
            u2[u] = U2[o];
            u3[u] = U3[o];
            rh[u] = X(j, r);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = r0 - u;
          if (r >= 0) {
            double v = (rh[u] - u2[u] * x1 - u3[u] * x2) * u1[u];
            if (fabs(v) > 1e150) {
              for (int q = 0; q < n; ++q) X(j, q) *= 1e-150;
#pragma unroll
              for (int w = 0; w < 8; ++w) rh[w] *= 1e-150;
              x1 *= 1e-150;
              x2 *= 1e-150;
              v *= 1e-150;
              ss *= 1e-300;
            }
            x2 = x1;
            x1 = v;
            X(j, r) = v;
            ss += v * v;
          }
        }
      }
      sc = 1.0 / sqrt(ss);
      if (it == 2 || maxpos > 0) {  // the last solve, or clusters to orthogonalise: scale now
        for (int r = 0; r < n; ++r) X(j, r) *= sc;
        sc = 1.0;
      }
    }
    __syncthreads();
    // vectors of one cluster: modified Gram-Schmidt in cluster order
    for (int pos = 1; pos <= maxpos; ++pos) {
      if (tid < kk && clus[2 * tid + 1] == pos) {
        const int j = tid;
        for (int j2 = clus[2 * j]; j2 < j; ++j2) {
          double dt = 0.0;
          for (int r = 0; r < n; ++r) dt += X(j2, r) * X(j, r);
          for (int r = 0; r < n; ++r) X(j, r) -= dt * X(j2, r);
        }
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += X(j, r) * X(j, r);
        s = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        for (int r = 0; r < n; ++r) X(j, r) *= s;
      }
      __syncthreads();
    }
  }
  // Cholesky QR of the vectors (their Gram is the identity to ~eps/gap
  // after inverse iteration; one pass leaves them orthonormal to ~eps).
  // Gram in U1 (free now); when it is the identity to 1e-12 the vectors
  // are kept as they are, else R^T R = Gram (right-looking, the workgroup
  // updating the trailing block per column) and the rows of X are
  // multiplied by R^-1 (reciprocal diagonal in U2).
  {
    double* Gq = U1;
    double* rinv = U2;
    double dev = 0.0;
    for (int e2 = tid; e2 < kk * kk; e2 += nt) {
      const int a = e2 / kk, b = e2 % kk;
      if (b < a) continue;
      double dt = 0.0;
      for (int r = 0; r < n; ++r) dt += X(a, r) * X(b, r);
      Gq[a * kk + b] = dt;
      Gq[b * kk + a] = dt;
      dev = fmax(dev, fabs(a == b ? dt - 1.0 : dt));
    }
    {
      int dummy = 0;
      block_argmax(dev, dummy, red, reinterpret_cast<int*>(part));
    }
    int ok = 1;
    if (dev > 1e-12) {
      for (int jj = 0; jj < kk; ++jj) {
        const double dg = Gq[jj * kk + jj];
        if (!(dg > 0.25)) {  // the same decision on every thread
          ok = 0;
          break;
        }
        const double rj = sqrt(dg), ir = 1.0 / rj;
        __syncthreads();  // every thread has read the pivot
        for (int c2 = jj + 1 + tid; c2 < kk; c2 += nt) Gq[jj * kk + c2] *= ir;
        if (tid == 0) {
          Gq[jj * kk + jj] = rj;
          rinv[jj] = ir;
        }
        __syncthreads();
        const int m2 = kk - jj - 1;
        for (int e2 = tid; e2 < m2 * m2; e2 += nt) {
          const int a = jj + 1 + e2 / m2, b = jj + 1 + e2 % m2;
          if (b >= a) Gq[a * kk + b] -= Gq[jj * kk + a] * Gq[jj * kk + b];
        }
        __syncthreads();
      }
      if (ok) {
        for (int r = tid; r < n; r += nt) {
          for (int j2 = 0; j2 < kk; ++j2) {
            double v = X(j2, r);
            for (int t2 = 0; t2 < j2; ++t2) v -= X(t2, r) * Gq[t2 * kk + j2];
            X(j2, r) = v * rinv[j2];
          }
        }
      }
    }
    if (tid == 0) s_busy = ok;
    __syncthreads();
  }
  // Rayleigh quotients y^T T y (scaled back)
  if (tid < kk) {
    const int j = tid;
    double s = 0.0, xm = 0.0, x0 = X(j, 0);
    for (int r = 0; r < n; ++r) {
      const double xp = r + 1 < n ? X(j, r + 1) : 0.0;
      double ty = d[r] * x0 + e[r] * xp;
      if (r > 0) ty += e[r - 1] * xm;
      s += x0 * ty;
      xm = x0;
      x0 = xp;
    }
    lam[j] = s * gmax;
  }
  __syncthreads();

  // ---- 4. back-transformation x = H_0 ... H_{n-3} y -------------------------------------
  t_inv = wall_clock64();
  // A group of gs lanes (a power of two, inside one wavefront) per vector;
  // lane sp of a group always owns the rows r = sp (mod gs), so the groups
  // share nothing and the partial dot products are summed with shuffles:
  // no barrier inside the loop.
  {
    int gs = 1;
    while (gs < 64 && 2 * gs * kk <= nt) gs *= 2;
    const int j = tid / gs, sp = tid % gs;
    for (int i = n - 3; i >= 0; --i) {
      const double ti = tau[i];
      if (ti == 0.0) continue;
      const int r0 = i + 1 + ((sp - (i + 1)) % gs + gs) % gs;
      double acc = 0.0;
      if (j < kk)
        for (int r = r0; r < n; r += gs) acc += (r == i + 1 ? 1.0 : W[int64_t(r) * n + i]) * X(j, r);
      for (int o = gs >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (j < kk) {
        const double sj = acc * ti;
        for (int r = r0; r < n; r += gs) X(j, r) -= sj * (r == i + 1 ? 1.0 : W[int64_t(r) * n + i]);
      }
    }
    __syncthreads();
  }
  for (int64_t x = tid; x < int64_t(n) * k; x += nt) {
    const int r = int(x / k), j = int(x % k);
    E[int64_t(r) * lde + j] = j < kk ? X(j, r) : 0.0;
  }
  __syncthreads();
  // after the Cholesky QR the vectors are orthonormal to ~eps and the
  // reflectors keep them so; the check (and CGS2) only without it
  if (!s_busy) {
    orthonormalize(E, n, kk, lde, 1, pw, red, &s_flag);
    if (cnt && tid == 0 && s_flag) cnt->fallbacks += 1;
  }
  };
  if (2 * kk < n) vectors(XinW{W, n});
  else vectors(XinT{U1 + int64_t(3) * n * kk, kk});
  if (cnt && tid == 0) {
    cnt->calls += 1;
    cnt->sweeps += uint64_t(iters + 1);
    cnt->values_ticks += t_bis - t_start;
    cnt->tail_ticks += wall_clock64() - t_bis;
    cnt->tri_ticks += t_tri - t_start;
    cnt->invit_ticks += t_inv - t_bis;
  }
  return lam;
}

// ---------------------------------------------------------------------------
// Warm-started leading eigenvectors
// ---------------------------------------------------------------------------

// Pair a (0 <= a < m / 2) of round t (0 <= t < m - 1) of a round-robin
// schedule over m (even) indices: index m - 1 meets t, and for a >= 1 the
// indices (t + a) and (t - a) modulo m - 1 meet, so every pair meets once
// per m - 1 rounds and the m / 2 pairs of a round are disjoint.
__device__ __forceinline__ void robin_pair(int t, int a, int m, int* p, int* q) {
  int x, y;
  if (a == 0) {
    x = t;
    y = m - 1;
  } else {
    x = (t + a) % (m - 1);
    y = (t - a + (m - 1)) % (m - 1);
  }
  *p = x < y ? x : y;
  *q = x < y ? y : x;
}

// Rows of Q = Y L^{-T} for the Cholesky factor L of Y^T Y (lower triangle of
// Lm, k x k; dinv[j] = 1 / L(j, j)): one row per lane, forward substitution
// column by column so each step's updates are independent; in registers for
// k <= 16, else in Q's row.
__device__ __forceinline__ void chol_solve_rows(const double* Y, double* Q, int n, int k, const double* Lm,
                                                const double* dinv) {
  constexpr int KM = 16;
  if (k > KM) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double* q = Q + int64_t(i) * k;
      for (int j = 0; j < k; ++j) q[j] = Y[int64_t(i) * k + j];
      for (int j = 0; j < k; ++j) {
        const double qj = q[j] * dinv[j];
        q[j] = qj;
        for (int t = j + 1; t < k; ++t) q[t] -= qj * Lm[t * k + j];
      }
    }
    __syncthreads();
    return;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double y[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) y[j] = j < k ? Y[int64_t(i) * k + j] : 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j < k) {
        const double qj = y[j] * dinv[j];
        y[j] = qj;
#pragma unroll
        for (int t = j + 1; t < KM; ++t)
          if (t < k) y[t] -= qj * Lm[t * k + j];
      }
    }
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) Q[int64_t(i) * k + j] = y[j];
  }
  __syncthreads();
}

// Leading k eigenvectors of a symmetric positive semidefinite n x n matrix
// S (a Gram; row-major, both triangles) from a start: E (n x k, row stride
// lde) holds orthonormal vectors close to them (the previous ALS sweep's
// for the same mode in the same coordinates, or a hit's own vectors).
//   * Block subspace iteration (Golub & Van Loan, Sec. 8.2.4): Y = S Q,
//     H = Q^T Y and the residual R = Y - Q H; until ||R||_F is at most
//     1e-11 max_j H(j, j), or the certificate below holds already with a
//     Gershgorin lower bound for min theta, Q becomes the Cholesky QR of Y.
//     From the third step on, the observed contraction of ||R|| predicts
//     the steps still needed to reach 1e-8 of the smallest diagonal entry
//     of H (the certificate's level) or 1e-11 of the largest; a start that
//     cannot converge within kWarmMaxSteps is given up early.
//   * Rayleigh-Ritz (Sec. 8.1.4): H = W Theta W^T by cyclic Jacobi (Sec.
//     8.5: the two-by-two symmetric Schur rotation, round-robin pairs, the
//     m / 2 disjoint rotations of a round applied together, each thread
//     updating whole 2 x 2 blocks in place), until no off-diagonal entry
//     exceeds 1e-12 sqrt(|H(p, p) H(q, q)|).
//   * A certificate that span Q is S's leading invariant subspace: in the
//     basis [Q, Q_perp], S = [[H, R'^T], [R', C]] with ||R'|| = ||R||, and
//     C is positive semidefinite, so lambda_max(C) <= min(trace C, ||C||_F)
//     with trace C = trace S - sum theta and ||C||_F^2 = ||S||_F^2 -
//     ||H||_F^2 - 2 ||R||_F^2 (rounding margins added).  By Weyl's theorem
//     S's eigenvalues lie within ||R|| of those of blockdiag(H, C), so
//     gap = min theta - that bound - 2 ||R|| > 0 makes S's top k the ones
//     near theta, and the sin-theta theorem bounds the angle between span Q
//     and the exact leading subspace by ||R|| / gap, required below 1e-8.
// On success the Ritz vectors Q W, in descending order of theta, replace E
// and it returns 1; otherwise E is untouched and it returns 0, or -1 when
// the refusal shows no gap after the k-th eigenvalue (a residual that
// contracts by less than half a step, or a converged subspace that fails
// the certificate): the caller then runs the full solver.  S is only read.  qy: 2 n k doubles
// (Q and Y), sm: warm_small_doubles(k) doubles (the k x k matrices, kept in
// LDS by the callers), k <= 32, n > k.
constexpr int kWarmMaxSteps = 10;
__device__ __forceinline__ int eig_top_warm(const double* S, int n, int k, double* E, int lde, double* qy,
                                            double* sm, double* red, EigCounters* cnt) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const uint64_t t_start = wall_clock64();
  double* Q = qy;
  double* Y = Q + int64_t(n) * k;
  double* H = sm;
  double* W = H + k * k;
  const int m = (k + 1) & ~1, hp = m / 2;
  double* cs = W + k * k;                            // c, s, t of each pair of a round
  int* pos = reinterpret_cast<int*>(cs + 3 * hp);    // output column of each Ritz vector
  int* flag = pos + k;                               // [1]: an off-diagonal entry left to rotate
  // |S|_F^2 and trace S for the certificate; Q = E
  double a2 = 0.0, tr = 0.0;
  for (int e = tid; e < n * n; e += nt) {
    const double v = S[e];
    a2 += v * v;
    if (e % (n + 1) == 0) tr += v;
  }
  const double nS2 = block_sum(a2, red);
  const double trS = block_sum(tr, red);
  for (int e = tid; e < n * k; e += nt) Q[e] = E[int64_t(e / k) * lde + e % k];
  __syncthreads();
  bool conv = false, nogap = false;
  double rho = 0.0, rho_prev = 0.0;
  int it = 0;
  for (;;) {
    ++it;
    gemm_f64(n, k, n, [&](int i, int c) { return S[int64_t(i) * n + c]; },
             [&](int c, int j) { return Q[int64_t(c) * k + j]; },
             [&](int i, int j, double v) { Y[int64_t(i) * k + j] = v; });
    gemm_f64(k, k, n, [&](int i, int c) { return Q[int64_t(c) * k + i]; },
             [&](int c, int j) { return Y[int64_t(c) * k + j]; }, [&](int i, int j, double v) { H[i * k + j] = v; });
    double part = 0.0;
    gemm_f64(n, k, k, [&](int i, int c) { return Q[int64_t(i) * k + c]; }, [&](int c, int j) { return H[c * k + j]; },
             [&](int i, int j, double v) {
               const double d = Y[int64_t(i) * k + j] - v;
               part += d * d;
             });
    rho = sqrt(block_sum(part, red));
    double hmax = 0.0, hmin = H[0];
    for (int j = 0; j < k; ++j) {
      hmax = fmax(hmax, H[j * k + j]);
      hmin = fmin(hmin, H[j * k + j]);
    }
    // Once near convergence, the certificate below with Gershgorin's lower
    // bound for the smallest eigenvalue of H (symmetrised) in place of the
    // exact one: when it already holds, this step's Q is final.
    bool cert = false;
    if (hmax > 0.0 && rho <= 1e-6 * hmax) {
      double nlb = -1e300, trp = 0.0, h2p = 0.0;
      for (int i = tid; i < k; i += nt) {
        double off = 0.0;
        for (int j = 0; j < k; ++j) {
          const double hs = 0.5 * (H[i * k + j] + H[j * k + i]);
          h2p += hs * hs;
          if (j != i) off += fabs(hs);
        }
        trp += H[i * k + i];
        nlb = fmax(nlb, off - H[i * k + i]);
      }
      const double lb = -block_max(nlb, red);
      const double trH = block_sum(trp, red), nH2 = block_sum(h2p, red);
      const double cT = fmax(0.0, trS - trH) + 1e-12 * fabs(trS);
      const double cF = sqrt(fmax(0.0, nS2 - nH2 - 2.0 * rho * rho) + 1e-12 * nS2);
      const double gap = lb - fmin(cT, cF) - 2.0 * rho;
      cert = gap > 0.0 && rho <= 1e-8 * gap;
    }
    __syncthreads();  // H is read; the Cholesky QR overwrites it
    if (!(hmax > 0.0)) break;
    if (cert || rho <= 1e-11 * hmax) {
      conv = true;
      break;
    }
    if (it >= kWarmMaxSteps) break;
    if (it >= 3) {  // steps still needed at the observed contraction (to the certificate's level)
      const double f = rho / rho_prev;
      const double target = fmax(1e-11 * hmax, 1e-8 * hmin);
      nogap = !(f < 0.5);
      if (nogap || double(it) + log(target / rho) / log(f) > double(kWarmMaxSteps)) break;
    }
    rho_prev = rho;
    // Cholesky QR: H <- Y^T Y = L L^T (lower triangle), Q <- Y L^{-T}
    gemm_f64(k, k, n, [&](int i, int c) { return Y[int64_t(c) * k + i]; },
             [&](int c, int j) { return Y[int64_t(c) * k + j]; }, [&](int i, int j, double v) { H[i * k + j] = v; });
    const double d0 = H[0];
    bool ok = true;
    for (int j = 0; j < k; ++j) {
      const double d = H[j * k + j];
      if (!(d > 1e-24 * d0)) {  // Y (numerically) rank deficient
        ok = false;
        break;
      }
      const double ljj = sqrt(d), inv = 1.0 / ljj;
      __syncthreads();  // every thread has read H(j, j)
      for (int i = j + 1 + tid; i < k; i += nt) H[i * k + j] *= inv;
      if (tid == 0) {
        H[j * k + j] = ljj;
        cs[j] = inv;
      }
      __syncthreads();
      const int mm = k - j - 1;
      for (int e = tid; e < mm * mm; e += nt) {
        const int i = j + 1 + e / mm, l = j + 1 + e % mm;
        if (l <= i) H[i * k + l] -= H[i * k + j] * H[l * k + j];
      }
      __syncthreads();
    }
    if (!ok) break;
    chol_solve_rows(Y, Q, n, k, H, cs);
  }
  bool accept = false;
  const uint64_t t_rr = wall_clock64();
  if (conv) {
    // Rayleigh-Ritz: H (symmetrised) = W Theta W^T by cyclic Jacobi
    for (int e = tid; e < k * k; e += nt) {
      const int i = e / k, j = e % k;
      W[e] = i == j ? 1.0 : 0.0;
      if (j > i) {
        const double v = 0.5 * (H[e] + H[j * k + i]);
        H[e] = v;
        H[j * k + i] = v;
      }
    }
    __syncthreads();
    // an entry calls for a rotation above 1e-12 of its diagonal's scale
    // (the relative criterion for positive definite Jacobi; the Ritz
    // vectors only order the basis, the subspace is fixed already)
    auto rotates = [](double hpq, double hpp, double hqq) {
      return hpq != 0.0 && fabs(hpq) > 1e-12 * sqrt(fabs(hpp) * fabs(hqq));
    };
    // whether some off-diagonal entry still calls for a rotation (flag[1];
    // the last barrier keeps the next clear behind every reader)
    auto off_diag = [&]() {
      if (tid == 0) flag[1] = 0;
      __syncthreads();
      for (int e = tid; e < k * k; e += nt) {
        const int i = e / k, j = e % k;
        const double v = H[e];
        if (j > i && rotates(v, H[i * k + i], H[j * k + j])) flag[1] = 1;
      }
      __syncthreads();
      const bool any = flag[1] != 0;
      __syncthreads();
      return any;
    };
    bool done = !off_diag();
    for (int sw = 0; sw < 12 && !done; ++sw) {
      for (int t = 0; t < m - 1; ++t) {
        for (int a = tid; a < hp; a += nt) {
          int p, q;
          robin_pair(t, a, m, &p, &q);
          double c = 1.0, sn = 0.0, tt = 0.0;
          if (q < k) {
            const double hpq = H[p * k + q], hpp = H[p * k + p], hqq = H[q * k + q];
            if (rotates(hpq, hpp, hqq)) {
              const double tau = (hqq - hpp) / (2.0 * hpq);
              tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + tt * tt);
              sn = tt * c;
            }
          }
          cs[3 * a] = c;
          cs[3 * a + 1] = sn;
          cs[3 * a + 2] = tt;
        }
        __syncthreads();
        // H <- J^T H J, block (pair a rows) x (pair b columns) per thread
        for (int u = tid; u < hp * hp; u += nt) {
          const int a = u / hp, b = u % hp;
          const double ca = cs[3 * a], sa = cs[3 * a + 1], cb = cs[3 * b], sb = cs[3 * b + 1];
          if (sa == 0.0 && sb == 0.0) continue;
          int p, q, p2, q2;
          robin_pair(t, a, m, &p, &q);
          robin_pair(t, b, m, &p2, &q2);
          if (a == b) {  // the rotated pair itself: exact diagonal, zero coupling
            const double tt = cs[3 * a + 2], hpq = H[p * k + q];
            H[p * k + p] -= tt * hpq;
            H[q * k + q] += tt * hpq;
            H[p * k + q] = 0.0;
            H[q * k + p] = 0.0;
            continue;
          }
          const bool qv = q < k, q2v = q2 < k;
          const double x00 = H[p * k + p2], x01 = q2v ? H[p * k + q2] : 0.0;
          const double x10 = qv ? H[q * k + p2] : 0.0, x11 = qv && q2v ? H[q * k + q2] : 0.0;
          const double r00 = ca * x00 - sa * x10, r01 = ca * x01 - sa * x11;  // J_a^T rows
          const double r10 = sa * x00 + ca * x10, r11 = sa * x01 + ca * x11;
          H[p * k + p2] = cb * r00 - sb * r01;  // then J_b columns
          if (q2v) H[p * k + q2] = sb * r00 + cb * r01;
          if (qv) H[q * k + p2] = cb * r10 - sb * r11;
          if (qv && q2v) H[q * k + q2] = sb * r10 + cb * r11;
        }
        for (int u = tid; u < k * hp; u += nt) {  // W <- W J
          const int i = u / hp, b = u % hp;
          const double cb = cs[3 * b], sb = cs[3 * b + 1];
          if (sb == 0.0) continue;
          int p2, q2;
          robin_pair(t, b, m, &p2, &q2);
          const double w0 = W[i * k + p2], w1 = W[i * k + q2];
          W[i * k + p2] = cb * w0 - sb * w1;
          W[i * k + q2] = sb * w0 + cb * w1;
        }
        __syncthreads();
      }
      done = !off_diag();
    }
    if (done) {
      double th_min = 0.0, s1 = 0.0, s2 = 0.0;
      for (int j = 0; j < k; ++j) {
        const double th = H[j * k + j];
        th_min = j == 0 ? th : fmin(th_min, th);
        s1 += th;
        s2 += th * th;
      }
      const double cT = fmax(0.0, trS - s1) + 1e-12 * fabs(trS);
      const double cF = sqrt(fmax(0.0, nS2 - s2 - 2.0 * rho * rho) + 1e-12 * nS2);
      const double gap = th_min - fmin(cT, cF) - 2.0 * rho;
      accept = gap > 0.0 && rho <= 1e-8 * gap;
      nogap = !accept;
    }
  }
  if (accept) {
    for (int j = tid; j < k; j += nt) {  // descending theta, ties by index
      const double th = H[j * k + j];
      int r = 0;
      for (int i = 0; i < k; ++i) {
        const double o = H[i * k + i];
        r += (o > th || (o == th && i < j)) ? 1 : 0;
      }
      pos[j] = r;
    }
    __syncthreads();
    gemm_f64(n, k, k, [&](int i, int c) { return Q[int64_t(i) * k + c]; }, [&](int c, int j) { return W[c * k + j]; },
             [&](int i, int j, double v) { E[int64_t(i) * lde + pos[j]] = v; });
  }
  if (cnt && tid == 0) {
    cnt->warm += accept ? 1 : 0;
    cnt->warm_fail += accept ? 0 : 1;
    cnt->warm_steps += uint64_t(it);
    const uint64_t t_end = wall_clock64();
    cnt->warm_ticks += t_end - t_start;
    cnt->warm_rr_ticks += t_end - t_rr;
  }
  __syncthreads();
  return accept ? 1 : (nogap ? -1 : 0);
}

// The eigensolver the kernels use.
__device__ __forceinline__ const double* eig_top(double* W, int n, int k, double* E, int lde, double* red,
                                                 double* tmp, EigCounters* cnt, double* vec,
                                                 double* lfree = nullptr, int64_t nfree = 0) {
  return eig_top_tri(W, n, k, E, lde, red, tmp, cnt, vec, lfree, nfree);
}

}  // namespace tk
