// Shared host/device definitions: dyadic tree topology, Recall, effective
// ranks, device views of the node store and job descriptors, and the
// workspace layout of a stitch job.  Everything here is compiled once for the
// host and once for the device from the same source, so the host-side hit
// sets and workspace sizes are bit-identical to what the kernels use.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#define TK_HD __host__ __device__ inline

namespace tk {

constexpr int MAXP = 7;      // modes handled by the kernels (time included)
constexpr int MAXLEV = 48;   // tree levels (2^47 leaf blocks)
constexpr int MAXHITS = 64;  // hits per query: <= 2(h-1) for trees of height <= 33
constexpr int EIG_MAXK_HOST = 1024;  // largest eigenproblem a job may need

// ---------------------------------------------------------------------------
// Topology.  The stream segment tree built by Alg. "append"/"insert" (Sec.
// 6.2) is the dyadic segment tree over leaf blocks, created lazily: node
// (k, j) covers blocks [j 2^k, (j+1) 2^k), exists once its first block has
// arrived, and is complete (a leaf or intermediate node) once its last block
// has.  The root after T_b blocks sits at level ceil(log2 T_b) (Thm.
// "alg-log-height": height ceil(log2 T) + 1).
// ---------------------------------------------------------------------------

TK_HD int root_level(int64_t Tb) {
  int k = 0;
  while ((int64_t(1) << k) < Tb) ++k;
  return k;
}

TK_HD bool node_complete(int k, int64_t j, int64_t Tb) { return ((j + 1) << k) <= Tb; }

TK_HD int popcount64(uint64_t x) {
  int c = 0;
  while (x) {
    x &= x - 1;
    ++c;
  }
  return c;
}

TK_HD int bitlen64(uint64_t x) {
  int c = 0;
  while (x) {
    x >>= 1;
    ++c;
  }
  return c;
}

// 1-based creation order of node (k, j) under Alg. "append"/"insert": the
// node is created when block c arrives, c = 2^(k-1) for a new root (j = 0,
// k >= 1) and c = j 2^k otherwise; blocks before c created
// [c>=1] + [c>=2](2(c-1) - popcount(c-1) + bitlen(c-1)) nodes; at block c the
// new root (if c is a power of two) comes first, then levels nu_2(c) .. 0.
TK_HD int64_t node_id(int k, int64_t j) {
  const int64_t c = (j == 0 && k >= 1) ? (int64_t(1) << (k - 1)) : (j << k);
  int64_t before = 0;
  if (c == 1) {
    before = 1;
  } else if (c >= 2) {
    const uint64_t m = uint64_t(c - 1);
    before = 1 + 2 * int64_t(m) - popcount64(m) + bitlen64(m);
  }
  int64_t pos = 0;
  if (c > 0) {
    const bool pow2 = (c & (c - 1)) == 0;
    if (j == 0 && k >= 1) {
      pos = 0;  // the new root
    } else {
      const int nu = bitlen64(uint64_t(c & -c)) - 1;
      pos = (pow2 ? 1 : 0) + (nu - k);
    }
  }
  return before + 1 + pos;
}

struct Hit {
  int32_t level;
  int32_t partial;
  int64_t index;
  int64_t a;  // clipped start inside the node, in slices
  int64_t l;  // clipped length
};

// Alg. "recall" (Sec. 5.1) on the dyadic tree, iteratively with an explicit
// stack.  A complete node v is taken when den |[ts,te) & v| >= num |v|
// (theta = num/den, exact integer test); a leaf that is reached is taken even
// below the threshold (it has no children).  Hits come out in time order.
// Returns the number of hits (writes at most cap of them), or -1 if the range
// is outside [0, Tb ell) or empty.
constexpr int RECALL_STACK = 2 * MAXLEV + 4;

// sk: RECALL_STACK int64 of scratch (the device passes LDS).
TK_HD int recall_with_stack(int64_t ts, int64_t te, int64_t Tb, int64_t ell, int64_t num, int64_t den,
                            Hit* out, int cap, int64_t* sk) {
  if (!(ts >= 0 && ts < te && te <= Tb * ell)) return -1;
  int sp = 0;
  const int K = root_level(Tb);
  sk[sp++] = (int64_t(K) << 56) | 0;  // (level << 56) | index
  int n = 0;
  while (sp > 0) {
    const int64_t e = sk[--sp];
    const int k = int(e >> 56);
    const int64_t j = e & ((int64_t(1) << 56) - 1);
    const int64_t sig = (j << k) * ell;
    const int64_t tau = ((j + 1) << k) * ell;
    const int64_t lo = ts > sig ? ts : sig;
    const int64_t hi = te < tau ? te : tau;
    if (node_complete(k, j, Tb) && (k == 0 || den * (hi - lo) >= num * (tau - sig))) {
      if (n < cap) {
        out[n].level = k;
        out[n].index = j;
        out[n].a = lo - sig;
        out[n].l = hi - lo;
        out[n].partial = (lo != sig || hi != tau) ? 1 : 0;
      }
      ++n;
      continue;
    }
    const int64_t mid = sig + (tau - sig) / 2;
    const int64_t left = (int64_t(k - 1) << 56) | (2 * j);
    const int64_t right = (int64_t(k - 1) << 56) | (2 * j + 1);
    if (te <= mid) {
      sk[sp++] = left;
    } else if (ts >= mid) {
      sk[sp++] = right;
    } else {
      sk[sp++] = right;  // popped after the left subtree: time order
      sk[sp++] = left;
    }
  }
  return n;
}

TK_HD int recall(int64_t ts, int64_t te, int64_t Tb, int64_t ell, int64_t num, int64_t den, Hit* out, int cap) {
  int64_t sk[RECALL_STACK];
  return recall_with_stack(ts, te, Tb, ell, num, den, out, cap, sk);
}

// The fixed-block hit set of [ts, te) at snapshot Tb (the flat partition of
// the paper's efficiency-accuracy comparison): every complete node of
// `level` (ell 2^level slices) overlapping the range, clipped to it, then
// Alg. "recall" on the part past the last complete node of that level.  In
// time order; writes at most cap hits and returns the number needed.
inline int fixed_block_hits(int64_t ts, int64_t te, int64_t Tb, int64_t ell, int level, int64_t num, int64_t den,
                            Hit* out, int cap) {
  const int64_t B = ell << level;
  const int64_t full_end = (Tb >> level) * B;
  int n = 0;
  for (int64_t j = ts / B; j * B < te && j * B < full_end; ++j, ++n) {
    if (n >= cap) continue;
    const int64_t lo = ts > j * B ? ts : j * B;
    const int64_t hi = te < (j + 1) * B ? te : (j + 1) * B;
    out[n] = Hit{level, (lo != j * B || hi != (j + 1) * B) ? 1 : 0, j, lo - j * B, hi - lo};
  }
  if (te > full_end) {
    Hit rest[MAXHITS];
    const int m = recall(ts > full_end ? ts : full_end, te, Tb, ell, num, den, rest, MAXHITS);
    for (int i = 0; i < m && i < MAXHITS; ++i, ++n)
      if (n < cap) out[n] = rest[i];
  }
  return n;
}

// Effective ranks of a len x D_1 x ... x D_{p-1} range: r_0 <= len,
// r_n <= D_n, and r_n <= prod_{m != n} r_m, iterated to a fixed point (a mode
// rank cannot exceed the product of the others).
TK_HD void effective_ranks(int p, int64_t len, const int64_t* D, const int32_t* r, int32_t* out) {
  out[0] = int32_t(r[0] < len ? r[0] : len);
  for (int n = 1; n < p; ++n) out[n] = int32_t(r[n] < D[n] ? r[n] : D[n]);
  bool changed = true;
  while (changed) {
    changed = false;
    for (int n = 0; n < p; ++n) {
      int64_t other = 1;
      for (int m = 0; m < p; ++m)
        if (m != n) other *= out[m];
      if (out[n] > other) {
        out[n] = int32_t(other);
        changed = true;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Device view of the node store.  Level k holds n_k node slots; node (k, j)
// has a dense core of prod(rk[k]) floats, factors D_n x rk[k][n] for n >= 1,
// and owns rows [j ell 2^k, (j+1) ell 2^k) of the level's temporal plane
// (row width rk[k][0]).  Addresses are arithmetic; nodes never move.
// ---------------------------------------------------------------------------
struct StoreView {
  int32_t p;
  int32_t nlev;
  int64_t ell;
  int64_t D[MAXP];  // D[0] unused
  int32_t rk[MAXLEV][MAXP];
  int64_t core_elems[MAXLEV];
  float* core[MAXLEV];
  float* fac[MAXLEV][MAXP];
  float* plane[MAXLEV];
};

TK_HD int64_t fac_elems(const StoreView& st, int k, int n) { return st.D[n] * st.rk[k][n]; }

// A stitch job: a range query or the merge of two children (Alg. "insert").
// A query job carries its range and the committed block count it was
// admitted at; the kernel runs Recall on them itself, and the host's plan of
// the same hit set only sizes the workspace (ws_bytes).
struct Job {
  int32_t kind;  // 0 query (Recall on the device), 1 merge, 2 query on host-planned hits
  int32_t s;     // hits
  int32_t hit0;  // first hit in the launch's hit array
  int32_t pretrim;  // 1: the trims' row Grams were summed by trim_gram_kernel into the workspace (TG)
  int64_t L;
  int64_t ts;        // query range [ts, ts + L)
  int64_t Tb;        // committed leaf blocks seen by the query
  int64_t ws_bytes;  // workspace planned for the job
  int32_t rq[MAXP];          // output effective ranks
  float* out_core;           // prod(rq) floats
  float* out_fac[MAXP];      // [0]: L x rq[0] rows; [n]: D_n x rq[n]
  double* stats;             // STAT_COUNT doubles (see STAT_*)
  int64_t ws_off;            // byte offset of the job's workspace
};

// A leaf job: Tucker-ALS of one raw block.
struct LeafJob {
  const float* X;     // ell x D_1 x ... x D_{p-1}
  int64_t block;      // leaf index
  double* stats;
  int64_t ws_off;
};

// Per-job statistics; STAT_STATUS is 0, or 1 when the kernel's Recall did
// not reproduce the planned hit set, 2 when the workspace plan was too small
// (the job then did nothing); STAT_PHASE.. hold device time per phase in microseconds
// (trims, bases, init, temporal TTM+Gram, temporal eigen, other TTM+Gram,
// other eigens, finalize); STAT_T0/STAT_T1 the job's start and end on the
// device's 100 MHz clock; STAT_EIG_FALLBACK counts eigensolves whose vectors
// needed the Gram-Schmidt fallback; STAT_EIG.. hold eigensolver calls, bisection steps,
// and microseconds computing eigenvalues and eigenvectors; STAT_EIG_TRI and
// STAT_EIG_INVIT the parts of those spent in tridiagonalisation and in
// inverse iteration; STAT_EIG_WARM.. the warm-started sweep eigensolves:
// accepted, refused (the full solver ran after them), their subspace
// iteration steps and microseconds, and the part of those microseconds
// spent in the Rayleigh-Ritz step and the certificate.
enum {
  STAT_FIT = 0, STAT_ERR = 1, STAT_NORM = 2, STAT_SWEEPS = 3, STAT_CONV = 4, STAT_HITS = 5, STAT_STATUS = 6,
  STAT_PHASE = 8, STAT_NPHASE = 8, STAT_EIG = 16, STAT_T0 = 20, STAT_T1 = 21, STAT_EIG_FALLBACK = 22,
  STAT_EIG_TRI = 23, STAT_EIG_INVIT = 24, STAT_EIG_WARM = 25, STAT_EIG_WARM_FAIL = 26, STAT_EIG_WARM_STEPS = 27,
  STAT_EIG_WARM_US = 28, STAT_EIG_WARM_RR_US = 29, STAT_COUNT = 30
};
// Entries of a query's profile (tk_last_query_profile, tk_batch_profile):
// STAT_PHASE .. STAT_EIG_WARM_RR_US.
constexpr int PROFILE_COUNT = STAT_EIG_WARM_RR_US + 1 - STAT_PHASE;

// Rows of a partial hit's temporal factor per chunk of the trim pass: each
// chunk's Gram is summed by one workgroup of trim_gram_kernel, and the stitch
// kernel adds the chunk Grams in chunk order.
constexpr int64_t TRIM_CHUNK = 1024;
TK_HD int64_t trim_chunks(int64_t l) { return (l + TRIM_CHUNK - 1) / TRIM_CHUNK; }

// One chunk of the trim pass: the Gram (FP64, both triangles) of rows
// [0, rows) of V (k floats per row) into out (k x k).
struct TrimChunk {
  const float* V;
  int64_t rows;
  double* out;
  int32_t k;
  int32_t pad;
};

// ---------------------------------------------------------------------------
// Workspace layout of a stitch job (bump allocation, 256-byte aligned), used
// by the host to size the workspace and by the kernel to find its buffers.
// ---------------------------------------------------------------------------
struct StitchLayout {
  int64_t Ht[MAXHITS];        // float k_i x R_i, partial hits only
  int64_t F[MAXHITS];         // double k_i x k_i, partial hits only
  int64_t A[MAXHITS];         // float sum_{n>=1} rq_n x r_i^(n), modes in order
  int64_t A64[MAXHITS];       // double, same shape as A
  int64_t F0[MAXHITS];        // double k_i x rq_0
  int64_t C[MAXP];            // float D_n x sr_n (q_n x sr_n used)
  int64_t C64[MAXP];          // double, same
  int64_t Fn[MAXP];           // double sr_n x sr_n (basis route only)
  int64_t Pd[MAXP];           // double D_n x rq_n  ([0]: sk x rq_0)
  int64_t Pf[MAXP];           // float  same
  int64_t Fh[MAXP];           // double sr_n x rq_n
  int64_t M;                  // float sk x Rhat_0
  int64_t K;                  // float max_n D_n Rhat_n
  int64_t WS;                 // float max_n sr_n Rhat_n (stacked W_i^(n))
  int64_t T1, T2;             // float tmax
  int64_t D1, D2;             // double tmax (init and final FP64 core)
  int64_t S;                  // double 32 x 32 (mode Gram of one core)
  int64_t G;                  // float prod(rq)
  int64_t G64;                // double prod(rq)
  int64_t TG;                 // double: per partial hit, ceil(l / TRIM_CHUNK) partial k x k Grams (pretrim only)
  int64_t TMP;                // double eig_tmp_doubles(neig) (eigensolver / Cholesky scratch)
  int64_t EIG;                // double eig_doubles(neig) (only when neig > n_lds)
  int64_t total;
  int32_t sr[MAXP];           // sum over hits of r_i^(n)
  int32_t qmax[MAXP];
  int32_t sk;                 // sum over hits of k_i
  int32_t neig;               // largest eigenproblem
  int64_t tmax;
};

TK_HD int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// gram_rows (a trim's Gram over many rows) splits the rows among at most
// GRAM_ROWS_TILES partial 4 x 4 tiles of 16 doubles, whatever the workgroup
// size; the layout reserves that much scratch (in D1).  ntiles <= 36 for
// ranks <= 32, so ntiles * split <= GRAM_ROWS_TILES.
constexpr int GRAM_ROWS_TILES = 64;
TK_HD int gram_rows_split(int ntiles, int nthreads, int max_parts = GRAM_ROWS_TILES) {
  const int cap = nthreads < max_parts ? nthreads : max_parts;
  const int s = cap / ntiles;
  return s > 0 ? s : 1;
}

// Doubles needed by the eigensolver for an n x n problem: the matrix, then
// eight vectors of n (tridiagonal, reflector coefficients, eigenvalues,
// work vectors, brackets) and 256 doubles of per-thread partial results.
// The vector part of an eigen buffer (tridiagonal, reflector scalars,
// eigenvalues, work vectors, brackets, workgroup partials): it can live in
// LDS when the n x n matrix part does not.  It is at least large enough for
// the small matrices of a warm-started eigensolve with up to WARM_SMALL_K
// vectors (eig_top_warm), which use the same place.
constexpr int64_t WARM_SMALL_K = 16;
TK_HD int64_t warm_small_doubles(int64_t k) { return 2 * k * k + 2 * k + 4; }
TK_HD int64_t eig_vec_doubles(int64_t n) {
  const int64_t v = 8 * n + 256, w = warm_small_doubles(WARM_SMALL_K);
  return v > w ? v : w;
}
TK_HD int64_t eig_doubles(int64_t n) { return n * n + eig_vec_doubles(n); }

// Scratch of the eigensolver besides its buffer (inverse-iteration LU
// factors and, when they do not fit in the matrix buffer, vectors: 4 n k
// doubles for k <= 32 wanted eigenvectors), also used as n x n scratch by
// the Cholesky steps.
TK_HD int64_t eig_tmp_doubles(int64_t n) { return n * (n > 4 * 32 ? n : 4 * 32); }

// The layout record itself occupies the head of the job's workspace.
TK_HD void stitch_layout(const StoreView& st, const Hit* hits, int s, const int32_t* rq,
                         int n_lds, StitchLayout* Lo, int pretrim = 0) {
  const int p = st.p;
  int64_t off = align256(int64_t(sizeof(StitchLayout)));
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align256(off + (bytes > 0 ? bytes : 0));
    return o;
  };
  int64_t Rhat[MAXP];
  for (int n = 0; n < p; ++n) {
    int64_t pr = 1;
    for (int m = 0; m < p; ++m)
      if (m != n) pr *= rq[m];
    Rhat[n] = pr;
  }
  Lo->sk = 0;
  for (int n = 0; n < p; ++n) Lo->sr[n] = 0;
  Lo->tmax = 1;
  int maxk = 0;
  for (int i = 0; i < s; ++i) {
    const int lev = hits[i].level;
    const int k = st.rk[lev][0];
    int64_t R = 1;
    for (int n = 1; n < p; ++n) R *= st.rk[lev][n];
    Lo->Ht[i] = hits[i].partial ? take(int64_t(k) * R * 4) : -1;
    Lo->F[i] = hits[i].partial ? take(int64_t(k) * k * 8) : -1;
    int64_t asz = 0;
    for (int n = 1; n < p; ++n) asz += int64_t(rq[n]) * st.rk[lev][n];
    Lo->A[i] = take(asz * 4);
    Lo->A64[i] = take(asz * 8);
    Lo->F0[i] = take(int64_t(k) * rq[0] * 8);
    Lo->sk += k;
    if (k > maxk) maxk = k;
    for (int n = 1; n < p; ++n) Lo->sr[n] += st.rk[lev][n];
    int64_t t = (k > rq[0] ? k : rq[0]);
    for (int n = 1; n < p; ++n) t *= (st.rk[lev][n] > rq[n] ? st.rk[lev][n] : rq[n]);
    if (t > Lo->tmax) Lo->tmax = t;
    if (int64_t(k) * k > Lo->tmax) Lo->tmax = int64_t(k) * k;  // R~ of a trim
  }
  int neig = maxk > Lo->sk ? maxk : Lo->sk;
  int64_t kmax = 0;
  for (int n = 1; n < p; ++n) {
    // reduced coordinates: q_n <= sr_n on the basis route, q_n = D_n otherwise
    Lo->qmax[n] = int32_t(st.D[n]);
    Lo->C[n] = take(int64_t(Lo->qmax[n]) * Lo->sr[n] * 4);
    Lo->C64[n] = take(int64_t(Lo->qmax[n]) * Lo->sr[n] * 8);
    Lo->Fn[n] = take(st.D[n] > Lo->sr[n] ? int64_t(Lo->sr[n]) * Lo->sr[n] * 8 : 0);
    Lo->Pd[n] = take(int64_t(Lo->qmax[n]) * rq[n] * 8);
    Lo->Pf[n] = take(int64_t(Lo->qmax[n]) * rq[n] * 4);
    Lo->Fh[n] = take(int64_t(Lo->sr[n]) * rq[n] * 8);
    if (Lo->sr[n] > neig) neig = Lo->sr[n];
    if (Lo->qmax[n] > neig) neig = Lo->qmax[n];
    const int64_t kn = int64_t(Lo->qmax[n]) * Rhat[n];
    if (kn > kmax) kmax = kn;
  }
  Lo->qmax[0] = Lo->sk;
  Lo->sr[0] = Lo->sk;
  Lo->Pd[0] = take(int64_t(Lo->sk) * rq[0] * 8);
  Lo->Pf[0] = take(int64_t(Lo->sk) * rq[0] * 4);
  Lo->M = take(int64_t(Lo->sk) * Rhat[0] * 4);
  Lo->K = take(kmax * 4);
  int64_t wmax = 0;
  for (int n = 1; n < p; ++n)
    if (int64_t(Lo->sr[n]) * Rhat[n] > wmax) wmax = int64_t(Lo->sr[n]) * Rhat[n];
  Lo->WS = take(wmax * 4);
  // the HOSVD init keeps C_i S_i (q x r) in D1
  int64_t tq = 0;
  for (int n = 1; n < p; ++n) {
    int64_t rmax = 0;
    for (int i = 0; i < s; ++i)
      if (st.rk[hits[i].level][n] > rmax) rmax = st.rk[hits[i].level][n];
    if (int64_t(Lo->qmax[n]) * rmax > tq) tq = int64_t(Lo->qmax[n]) * rmax;
  }
  if (tq > Lo->tmax) Lo->tmax = tq;
  // partial Gram tiles of a trim (gram_rows): at most GRAM_ROWS_TILES x 16 doubles
  if (Lo->tmax < GRAM_ROWS_TILES * 16) Lo->tmax = GRAM_ROWS_TILES * 16;
  Lo->T1 = take(Lo->tmax * 4);
  Lo->T2 = take(Lo->tmax * 4);
  Lo->D1 = take(Lo->tmax * 8);
  Lo->D2 = take(Lo->tmax * 8);
  Lo->S = take(32 * 32 * 8);
  int64_t gel = 1;
  for (int n = 0; n < p; ++n) gel *= rq[n];
  Lo->G = take(gel * 4);
  Lo->G64 = take(gel * 8);
  Lo->neig = neig;
  int64_t tg = 0;
  if (pretrim)
    for (int i = 0; i < s; ++i)
      if (hits[i].partial) tg += trim_chunks(hits[i].l) * int64_t(st.rk[hits[i].level][0]) * st.rk[hits[i].level][0];
  Lo->TG = pretrim ? take(tg * 8) : -1;
  Lo->TMP = take(eig_tmp_doubles(neig) * 8);
  Lo->EIG = neig > n_lds ? take(eig_doubles(neig) * 8) : -1;
  Lo->total = off;
}

// Whether a stitch works on mode n in the coordinates of an orthonormal
// basis of the pieces' factor spans (sr_n concatenated columns of length
// D_n): when sr_n < pct% of D_n, i.e. when that shrinks the mode's
// eigenproblems enough to pay for the basis (a pivoted Cholesky
// factorisation and a triangular inverse of sr_n steps each); otherwise the
// D_n-dimensional coordinates are used as they are.
TK_HD bool span_basis(int sr, int64_t D, int pct) { return 100 * int64_t(sr) < int64_t(pct) * D; }

// Largest eigenproblem of a stitch job: the temporal one (sk) and, per mode,
// the reduced coordinates (q_n <= sr_n on the basis route, else D_n).  A
// basis found rank-deficient falls back to D_n; that rare case keeps all
// of its eigen buffer in the job's workspace.  Cholesky factorisations of
// the trims and bases need no vector part.
TK_HD int stitch_eig_need(const StitchLayout& lo, const StoreView& st, int pct) {
  int n = lo.sk;
  for (int m = 1; m < st.p; ++m) {
    const int e = span_basis(lo.sr[m], st.D[m], pct) ? lo.sr[m] : int(st.D[m]);
    if (e > n) n = e;
  }
  return n;
}

// How a leaf is decomposed.  Tucker-ALS on the raw block in general.  A leaf
// of one slice of a three-way series has temporal rank one and equal
// non-temporal ranks, and Tucker-ALS on it reaches the slice's truncated
// SVD (Eckart-Young), which is computed directly: from one eigensolve of
// the smaller side's Gram while that side has at most kSliceGramMax rows,
// else (1000 x 1000 slices, say) by block subspace iteration on that Gram,
// never formed, with slice_block(n, r) columns.
enum { LEAF_ALS = 0, LEAF_SLICE_GRAM = 1, LEAF_SLICE_ITER = 2 };
constexpr int kSliceGramMax = 256;
constexpr int kSliceIterMaxRank = 24;  // r + 8 <= 32 columns, the eigensolver's vector limit
constexpr int kSliceIterMax = 300;     // subspace iteration steps (a slice with no spectral gap)
TK_HD int slice_block(int64_t n, int r) {
  const int b = r <= 8 ? 16 : 32;
  return n < b ? int(n) : b;
}
TK_HD int leaf_route(const StoreView& st) {
  const int32_t* rq = st.rk[0];
  if (!(st.p == 3 && st.ell == 1 && rq[0] == 1 && rq[1] == rq[2])) return LEAF_ALS;
  const int64_t n = st.D[1] < st.D[2] ? st.D[1] : st.D[2];
  return n > kSliceGramMax && rq[1] <= kSliceIterMaxRank ? LEAF_SLICE_ITER : LEAF_SLICE_GRAM;
}

// Workspace of a leaf job.
struct LeafLayout {
  int64_t Ud[MAXP];  // double D_n x rq_n (D_0 = ell)
  int64_t Uf[MAXP];  // float
  int64_t T1, T2;    // float, size of the raw block
  int64_t V;         // double N x rq (other-side route)
  int64_t G;         // float prod(rq)
  int64_t TMP;       // double eig_tmp_doubles(neig) (eigensolver scratch)
  int64_t EIG;       // double eig_doubles(neig) when neig > n_lds
  // subspace iteration (LEAF_SLICE_ITER), doubles: Q, S Q, Q W, S Q W
  // (n x b each, n the smaller side), X^T Q (m x b), W (b x b)
  int64_t SQ, SY, SQW, SYW, SZ, SW;
  int64_t total;
  int32_t neig;
  int32_t route;
};

TK_HD void leaf_layout(const StoreView& st, int n_lds, LeafLayout* Lo) {
  const int p = st.p;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align256(off + (bytes > 0 ? bytes : 0));
    return o;
  };
  Lo->route = leaf_route(st);
  Lo->SQ = Lo->SY = Lo->SQW = Lo->SYW = Lo->SZ = Lo->SW = -1;
  if (Lo->route == LEAF_SLICE_ITER) {
    const int64_t n = st.D[1] < st.D[2] ? st.D[1] : st.D[2];
    const int64_t m = st.D[1] < st.D[2] ? st.D[2] : st.D[1];
    const int r = st.rk[0][1];
    const int b = slice_block(n, r);
    Lo->Ud[0] = take(8);
    Lo->Uf[0] = take(4);
    for (int k = 1; k < 3; ++k) {
      Lo->Ud[k] = take(st.D[k] * r * 8);
      Lo->Uf[k] = take(st.D[k] * r * 4);
    }
    Lo->T1 = Lo->T2 = Lo->V = -1;
    Lo->G = take(int64_t(r) * r * 4);
    Lo->SQ = take(n * b * 8);
    Lo->SY = take(n * b * 8);
    Lo->SQW = take(n * b * 8);
    Lo->SYW = take(n * b * 8);
    Lo->SZ = take(m * b * 8);
    Lo->SW = take(int64_t(b) * b * 8);
    Lo->neig = b;
    Lo->TMP = take(eig_tmp_doubles(b) * 8);
    Lo->EIG = b > n_lds ? take(eig_doubles(b) * 8) : -1;
    Lo->total = off;
    return;
  }
  int64_t Dm[MAXP];
  Dm[0] = st.ell;
  for (int n = 1; n < p; ++n) Dm[n] = st.D[n];
  int64_t size = 1;
  for (int n = 0; n < p; ++n) size *= Dm[n];
  const int32_t* rq = st.rk[0];
  int neig = 0;
  int64_t vmax = 0;
  for (int n = 0; n < p; ++n) {
    Lo->Ud[n] = take(Dm[n] * rq[n] * 8);
    Lo->Uf[n] = take(Dm[n] * rq[n] * 4);
    // HOSVD: mat_n(X) is D_n x size/D_n; sweeps: D_n x prod_{m != n} rq_m
    int64_t other = 1;
    for (int m = 0; m < p; ++m)
      if (m != n) other *= rq[m];
    const int64_t other0 = size / Dm[n];
    const int64_t e1 = Dm[n] < other0 ? Dm[n] : other0;
    const int64_t e2 = Dm[n] < other ? Dm[n] : other;
    if (e1 > neig) neig = int(e1);
    if (e2 > neig) neig = int(e2);
    if (Dm[n] > other0 && other0 * rq[n] > vmax) vmax = other0 * rq[n];
    if (Dm[n] > other && other * rq[n] > vmax) vmax = other * rq[n];
  }
  Lo->T1 = take(size * 4);
  Lo->T2 = take(size * 4);
  Lo->V = take(vmax * 8);
  int64_t gel = 1;
  for (int n = 0; n < p; ++n) gel *= rq[n];
  Lo->G = take(gel * 4);
  Lo->neig = neig;
  Lo->TMP = take(eig_tmp_doubles(neig) * 8);
  Lo->EIG = neig > n_lds ? take(eig_doubles(neig) * 8) : -1;
  Lo->total = off;
}

// Tucker-ALS from scratch on a raw range (the paper's accuracy reference
// and naive baseline): X holds L slices, C order.
struct RawJob {
  const float* X;
  int64_t L;
  int32_t rq[MAXP];
  float* out_core;
  float* out_fac[MAXP];
  double* stats;
  int64_t ws_off;
};

// Largest intermediate of the projections X x_{m != skip} U_m^T (every skip,
// and the core), taking modes in the order of the block kernels: the largest
// D_m / r_m reduction first.
TK_HD int64_t projection_max_elems(int p, const int32_t* Dm, const int32_t* rq) {
  int64_t best = 0;
  for (int skip = -1; skip < p; ++skip) {
    int64_t dims[MAXP];
    bool done[MAXP];
    for (int m = 0; m < p; ++m) {
      dims[m] = Dm[m];
      done[m] = false;
    }
    for (int step = 0; step < p; ++step) {
      int pick = -1;
      double ratio = 0.0;
      for (int m = 0; m < p; ++m) {
        if (m == skip || done[m]) continue;
        const double r = double(Dm[m]) / double(rq[m]);
        if (pick < 0 || r > ratio) {
          pick = m;
          ratio = r;
        }
      }
      if (pick < 0) break;
      done[pick] = true;
      dims[pick] = rq[pick];
      int64_t e = 1;
      for (int m = 0; m < p; ++m) e *= dims[m];
      if (e > best) best = e;
    }
  }
  return best;
}

// Workspace of a raw-range job (LeafLayout fields): factors, two projection
// buffers, the other-side vectors, the core and the eigen scratch.  The
// HOSVD initialises modes 1..p-1 only (the sweep starts with mode 0), so no
// Gram of the L x L side is formed.
TK_HD void raw_layout(int p, const int32_t* Dm, const int32_t* rq, int n_lds, LeafLayout* Lo) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align256(off + (bytes > 0 ? bytes : 0));
    return o;
  };
  int64_t size = 1;
  for (int n = 0; n < p; ++n) size *= Dm[n];
  int neig = 0;
  int64_t vmax = 0;
  for (int n = 0; n < p; ++n) {
    Lo->Ud[n] = take(int64_t(Dm[n]) * rq[n] * 8);
    Lo->Uf[n] = take(int64_t(Dm[n]) * rq[n] * 4);
    int64_t other = 1;
    for (int m = 0; m < p; ++m)
      if (m != n) other *= rq[m];
    const int64_t other0 = size / Dm[n];
    if (n > 0) {
      const int64_t e1 = Dm[n] < other0 ? Dm[n] : other0;
      if (e1 > neig) neig = int(e1);
      if (Dm[n] > other0 && other0 * rq[n] > vmax) vmax = other0 * rq[n];
    }
    const int64_t e2 = Dm[n] < other ? Dm[n] : other;
    if (e2 > neig) neig = int(e2);
    if (Dm[n] > other && other * rq[n] > vmax) vmax = other * rq[n];
  }
  const int64_t tsz = projection_max_elems(p, Dm, rq);
  Lo->T1 = take(tsz * 4);
  Lo->T2 = take(tsz * 4);
  Lo->V = take(vmax * 8);
  int64_t gel = 1;
  for (int n = 0; n < p; ++n) gel *= rq[n];
  Lo->G = take(gel * 4);
  Lo->neig = neig;
  Lo->TMP = take(eig_tmp_doubles(neig) * 8);
  Lo->EIG = neig > n_lds ? take(eig_doubles(neig) * 8) : -1;
  Lo->route = LEAF_ALS;
  Lo->SQ = Lo->SY = Lo->SQW = Lo->SYW = Lo->SZ = Lo->SW = -1;
  Lo->total = off;
}

}  // namespace tk
