// Drives the autotuner's search control (tk_tune_search.hpp) against a
// simulated clock: every candidate has a known cost per execution, the
// "device" advances the clock by it, and the search must keep the
// budget, abandon hopeless candidates after their warm-up, and find the
// cheapest candidate when the budget allows.  Prints "ok" or the failure.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tk_tune_search.hpp"

namespace {

struct Outcome {
  double elapsed = 0.0;
  double best = 1e300;
  int started = 0;
  int abandoned = 0;
};

// One search over costs_s (seconds per execution), reps timed executions
// after one warm-up; the clock also charges setup_s per candidate.
Outcome run(const std::vector<double>& costs_s, int reps, tk::TuneLimits lim, double setup_s) {
  tk::TuneSearch s(lim, 0.0);
  Outcome o;
  double now = 0.0;
  for (double c : costs_s) {
    if (!s.open(now)) break;
    ++o.started;
    now += setup_s + c;  // warm-up
    const double warm_ms = 1000.0 * c;
    if (!s.worth_timing(warm_ms)) {
      s.record(warm_ms, true, "sim", now);
      ++o.abandoned;
      continue;
    }
    now += reps * c;
    s.record(1000.0 * c, false, "sim", now);
  }
  o.elapsed = now;
  o.best = s.best_ms();
  return o;
}

int fails = 0;
void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what);
    ++fails;
  }
}

}  // namespace

int main() {
  // a many-mode grid: 112 candidates, the good ones at ~0.14 s per batch,
  // the narrow ones (64 threads on 5^7-element cores) 4x to 8x slower
  std::vector<double> costs;
  for (int i = 0; i < 112; ++i) {
    const bool narrow = (i % 4) < 2;
    costs.push_back(narrow ? 0.14 * (4.0 + 4.0 * ((i * 37) % 11) / 10.0) : 0.14 * (1.0 + 0.01 * ((i * 13) % 7)));
  }
  double cheapest = 1e300, total = 0.0;
  for (double c : costs) {
    cheapest = std::fmin(cheapest, 1000.0 * c);
    total += 2.0 * c + 0.02;
  }
  // the old search: no cap, no budget
  tk::TuneLimits none;
  none.budget_s = 0.0;
  none.cap = 0.0;
  const Outcome a = run(costs, 1, none, 0.02);
  check(std::fabs(a.elapsed - total) < 1e-9 && a.started == 112 && a.abandoned == 0, "unlimited search runs all");
  check(a.elapsed > 60.0, "the unlimited many-mode grid takes minutes");
  // cap only: narrow candidates are dropped after one execution
  tk::TuneLimits cap;
  cap.budget_s = 0.0;
  cap.cap = 3.0;
  const Outcome b = run(costs, 1, cap, 0.02);
  check(b.best == cheapest, "cap keeps the cheapest");
  check(b.abandoned >= 50, "cap abandons the slow half");
  check(b.elapsed < a.elapsed * 0.75, "cap saves time");
  // budget: no candidate starts after the budget; the overrun is at most one candidate
  tk::TuneLimits bud;
  bud.budget_s = 10.0;
  bud.cap = 3.0;
  const Outcome c = run(costs, 1, bud, 0.02);
  double worst = 0.0;
  for (double x : costs) worst = std::fmax(worst, 2.0 * x + 0.02);
  check(c.elapsed <= bud.budget_s + worst + 1e-9, "budget bounds the search");
  check(c.started < 112 && c.started > 0, "budget stops early");
  check(c.best < 1e300, "a budget-limited search still has a best");
  // a budget larger than the search changes nothing
  tk::TuneLimits big;
  big.budget_s = 1e6;
  big.cap = 3.0;
  const Outcome d = run(costs, 1, big, 0.02);
  check(d.started == 112 && d.best == b.best && d.abandoned == b.abandoned, "a large budget is no limit");
  // the first candidate is never abandoned, whatever it costs
  const Outcome e = run({5.0, 0.1, 0.2}, 1, cap, 0.0);
  check(e.abandoned == 0 && e.best == 100.0, "first candidate always timed");
  // abandoned candidates never become the best
  const Outcome f = run({0.1, 0.5, 0.05}, 1, cap, 0.0);
  check(f.abandoned == 1 && std::fabs(f.best - 50.0) < 1e-9, "abandoned candidate is skipped, later cheaper one wins");
  if (fails == 0) std::printf("ok\n");
  return fails == 0 ? 0 : 1;
}
