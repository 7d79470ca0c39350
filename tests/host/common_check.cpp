// Host-side checks of the shared tree/plan header (tk_common.hpp), built
// for the host only under AddressSanitizer and UndefinedBehaviorSanitizer:
// Recall and the fixed-block hit sets over every range of small trees
// (hits tile the range in time order, the hit-count bound of Alg. "recall"
// holds, no stack or buffer overrun), node ids (creation order: a
// permutation of 1..nodes), effective ranks (fixed point, bounds) and
// stitch workspace layouts (aligned, in bounds, in order).  Prints "ok" or
// the failures.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "tk_common.hpp"

using namespace tk;

static int fails = 0;
#define CHECK(c, ...)                   \
  do {                                  \
    if (!(c)) {                         \
      if (fails < 20) {                 \
        std::printf("FAIL %s: ", #c);   \
        std::printf(__VA_ARGS__);       \
        std::printf("\n");              \
      }                                 \
      ++fails;                          \
    }                                   \
  } while (0)

static void check_hits(const Hit* h, int n, int64_t ts, int64_t te, int64_t ell, const char* what) {
  int64_t t = ts;
  for (int i = 0; i < n; ++i) {
    const int64_t sig = (h[i].index << h[i].level) * ell;
    const int64_t tau = ((h[i].index + 1) << h[i].level) * ell;
    CHECK(sig + h[i].a == t, "%s [%ld,%ld) hit %d starts at %ld, expected %ld", what, long(ts), long(te), i,
          long(sig + h[i].a), long(t));
    CHECK(h[i].l > 0 && sig + h[i].a + h[i].l <= tau, "%s hit %d outside its node", what, i);
    CHECK(h[i].partial == ((h[i].a != 0 || h[i].l != tau - sig) ? 1 : 0), "%s partial flag", what);
    t += h[i].l;
  }
  CHECK(t == te, "%s [%ld,%ld) covered up to %ld", what, long(ts), long(te), long(t));
}

int main() {
  const int64_t thetas[][2] = {{1, 2}, {7, 10}, {9, 10}, {1, 1}};
  Hit hits[MAXHITS];
  for (int64_t ell : {1, 3}) {
    for (int64_t Tb = 1; Tb <= 70; ++Tb) {
      const int h = root_level(Tb) + 1;
      for (auto& th : thetas) {
        for (int64_t ts = 0; ts < Tb * ell; ++ts)
          for (int64_t te = ts + 1; te <= Tb * ell; ++te) {
            const int n = recall(ts, te, Tb, ell, th[0], th[1], hits, MAXHITS);
            CHECK(n >= 1 && n <= (h > 1 ? 2 * (h - 1) : 1), "recall count %d (height %d)", n, h);
            check_hits(hits, n, ts, te, ell, "recall");
            for (int level = 0; (int64_t(1) << level) <= Tb; ++level) {
              const int m = fixed_block_hits(ts, te, Tb, ell, level, th[0], th[1], hits, MAXHITS);
              // more than MAXHITS blocks: the count is returned (the caller refuses the range)
              CHECK(m >= 1, "fixed-block count %d", m);
              if (m <= MAXHITS) check_hits(hits, m, ts, te, ell, "fixed");
            }
          }
      }
      CHECK(recall(0, 0, Tb, ell, 7, 10, hits, MAXHITS) == -1, "empty range refused");
      CHECK(recall(0, Tb * ell + 1, Tb, ell, 7, 10, hits, MAXHITS) == -1, "range past T refused");
    }
  }
  // node ids: every complete node of a tree of Tb blocks gets a distinct id in 1..nodes
  for (int64_t Tb = 1; Tb <= 300; ++Tb) {
    std::set<int64_t> ids;
    int64_t nodes = 0;
    for (int k = 0; (int64_t(1) << k) <= Tb; ++k)
      for (int64_t j = 0; node_complete(k, j, Tb); ++j) {
        ids.insert(node_id(k, j));
        ++nodes;
      }
    CHECK(int64_t(ids.size()) == nodes && *ids.begin() >= 1, "node ids distinct for Tb=%ld", long(Tb));
  }
  // effective ranks
  const int64_t D[MAXP] = {0, 20, 3, 5, 7, 2, 9};
  for (int p = 2; p <= MAXP; ++p)
    for (int64_t len = 1; len <= 40; ++len)
      for (int r = 1; r <= 25; r += 3) {
        int32_t rq[MAXP], out[MAXP];
        for (int n = 0; n < p; ++n) rq[n] = r;
        effective_ranks(p, len, D, rq, out);
        for (int n = 0; n < p; ++n) {
          int64_t other = 1;
          for (int m = 0; m < p; ++m)
            if (m != n) other *= out[m];
          CHECK(out[n] >= 1 && out[n] <= rq[n] && out[n] <= other && (n ? out[n] <= D[n] : out[n] <= len),
                "effective rank p=%d len=%ld", p, long(len));
        }
      }
  // stitch workspace layouts for the hit sets of every range of a small tree
  StoreView st{};
  st.p = 3;
  st.ell = 2;
  st.D[1] = 12;
  st.D[2] = 9;
  st.nlev = 8;
  const int32_t rr[MAXP] = {5, 5, 4};
  for (int k = 0; k < st.nlev; ++k) {
    const int32_t* r = rr;
    int32_t out[MAXP];
    effective_ranks(st.p, st.ell << k, st.D, r, out);
    int64_t ce = 1;
    for (int n = 0; n < st.p; ++n) {
      st.rk[k][n] = out[n];
      ce *= out[n];
    }
    st.core_elems[k] = ce;
  }
  for (int64_t Tb = 1; Tb <= 64; ++Tb)
    for (int64_t ts = 0; ts < Tb * st.ell; ts += 3)
      for (int64_t te = ts + 1; te <= Tb * st.ell; te += 5) {
        const int n = recall(ts, te, Tb, st.ell, 7, 10, hits, MAXHITS);
        int32_t rq[MAXP];
        effective_ranks(st.p, te - ts, st.D, rr, rq);
        for (int n_lds : {0, 32, 96}) {
          StitchLayout lo;
          stitch_layout(st, hits, n, rq, n_lds, &lo);
          std::vector<int64_t> offs;
          for (int i = 0; i < n; ++i) {
            offs.push_back(lo.A[i]);
            offs.push_back(lo.A64[i]);
            offs.push_back(lo.F0[i]);
            if (hits[i].partial) {
              offs.push_back(lo.Ht[i]);
              offs.push_back(lo.F[i]);
            }
          }
          for (int m = 1; m < st.p; ++m)
            for (int64_t o : {lo.C[m], lo.C64[m], lo.Pd[m], lo.Pf[m], lo.Fh[m]}) offs.push_back(o);
          for (int64_t o : {lo.Pd[0], lo.Pf[0], lo.M, lo.K, lo.WS, lo.T1, lo.T2, lo.D1, lo.D2, lo.S, lo.G, lo.G64,
                            lo.TMP})
            offs.push_back(o);
          for (int64_t o : offs)
            CHECK(o >= int64_t(sizeof(StitchLayout)) && o < lo.total && o % 256 == 0, "layout offset %ld of %ld",
                  long(o), long(lo.total));
          CHECK(lo.sk >= 1 && lo.neig >= lo.sk, "layout sizes");
        }
      }
  if (fails == 0) std::printf("ok\n");
  return fails ? 1 : 0;
}
