// Sub-increment controller for adaptive load stepping (host only, no HIP).
//
// The paper fixes the load increments and names adaptive time stepping as the remedy for
// increments that need many Newton iterations (Sec. 4).  A load increment k -> k+1 is
// walked here in fractions theta of its length: the prescribed values move linearly from
// those of increment k to those of increment k+1.  A sub-increment that fails (Newton or
// CG cap, CG breakdown, det F <= 0) is retried from its starting state with half the
// fraction; one that converges within `grow_below` Newton iterations doubles the next
// fraction (never beyond what is left of the increment).
#pragma once

#include <algorithm>

namespace ghom {

struct SubstepClock {
  double theta = 0.0;   // completed fraction of the increment
  double dtheta = 1.0;  // length of the next sub-increment
  int cuts = 0;         // retries so far
  int max_cuts = 0;
  int grow_below = 0;

  SubstepClock(int max_cuts_, int grow_below_, double start_fraction)
      : dtheta(std::min(1.0, std::max(start_fraction, 0.0) > 0.0 ? start_fraction : 1.0)),
        max_cuts(max_cuts_),
        grow_below(grow_below_) {}

  bool done() const { return theta >= 1.0; }

  // end of the next sub-increment; exactly 1 when the rest of the increment fits, so the
  // last sub-increment lands on the increment's prescribed values without round-off
  double next_end() const { return dtheta >= 1.0 - theta ? 1.0 : theta + dtheta; }

  void accept(int newton_iters) {
    const double end = next_end();
    const double used = end - theta;
    theta = end;
    dtheta = used;
    if (newton_iters <= grow_below) dtheta = std::min(1.0, 2.0 * used);
  }

  // false when the cut budget is spent (the caller gives up)
  bool reject() {
    if (cuts >= max_cuts) return false;
    ++cuts;
    dtheta = 0.5 * (next_end() - theta);
    return true;
  }
};

// value at fraction t of the way from a to b (t == 1 gives b exactly)
inline void lerp9(const double* a, const double* b, double t, double* out) {
  for (int i = 0; i < 9; ++i) out[i] = t >= 1.0 ? b[i] : a[i] + t * (b[i] - a[i]);
}

}  // namespace ghom
