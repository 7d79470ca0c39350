// Search control of the launch autotuner (tk_autotune): time budget,
// early abandonment of slow candidates and progress lines.  Plain C++ (no
// HIP), so that the control logic can be exercised on the host against a
// simulated clock.
//
// Every candidate tuning is first run once (the warm-up, which also
// absorbs one-off costs).  A candidate whose warm-up already takes more
// than `cap` times the best mean so far cannot win and is not timed
// further; its warm-up time stands as its score.  Once `budget_s` seconds
// have passed since the search began, no new candidate is started (the
// one running finishes), and the search returns the best so far.
#pragma once

#include <cstdio>
#include <vector>

namespace tk {

struct TuneLimits {
  double budget_s = 60.0;  // wall-clock seconds for the whole search (<= 0: no limit)
  double cap = 3.0;        // abandon a candidate whose warm-up exceeds cap x best (<= 1: never)
  int progress = 0;        // 1: one line per candidate on stderr
};

class TuneSearch {
 public:
  TuneSearch(const TuneLimits& lim, double t0_s) : lim_(lim), t0_(t0_s) {}

  // May another candidate start at time now_s?
  bool open(double now_s) const { return !(lim_.budget_s > 0.0 && now_s - t0_ >= lim_.budget_s); }

  // After the warm-up run of a candidate: time it further?
  bool worth_timing(double warm_ms) const {
    return !(lim_.cap > 1.0 && best_ms_ < 1e300 && warm_ms > lim_.cap * best_ms_);
  }

  // Record a candidate's score (mean of its timed runs, or its warm-up time
  // when abandoned); returns true when it is the best so far.
  bool record(double ms, bool abandoned, const char* what, double now_s) {
    ++count_;
    if (abandoned) ++abandoned_;
    const bool best = !abandoned && ms < best_ms_;
    if (best) best_ms_ = ms;
    if (lim_.progress)
      std::fprintf(stderr, "[tk_autotune] %d: %s %.3f ms%s%s (%.1f s)\n", count_, what, ms,
                   abandoned ? " (abandoned after warm-up)" : "", best ? " best" : "", now_s - t0_);
    return best;
  }

  double best_ms() const { return best_ms_; }
  int count() const { return count_; }
  int abandoned() const { return abandoned_; }

 private:
  TuneLimits lim_;
  double t0_;
  double best_ms_ = 1e300;
  int count_ = 0;
  int abandoned_ = 0;
};

}  // namespace tk
