// Stopping rule of the conjugate-gradient solve, shared by the device kernel that ends each
// iteration and the host tests (constexpr, so it is usable in device code; no HIP).
//
// After an iteration that left the residual with r.r = rr:
//   converged  when rr <= thresh (the voxel-averaged L2 norm of Sec. 4 at or below its
//              threshold: thresh = tol^2 N);
//   cap        when the iteration count reaches max_it;
//   stalled    when rr has not gone below the smallest value seen in the solve for
//              kCgStallWindow iterations in a row.
// A stall is what conjugate gradients show when the right-hand side has a component the
// operator cannot reach (a near-null direction, e.g. a rigid rotation under full stress
// control) or when float32 round-off floors the residual above the threshold.  On healthy
// solves of the benchmark workloads the residual reaches a new minimum at every iteration or
// every other one, so the window costs a stalled solve about twenty iterations and never
// cuts a healthy one.  The caller continues Newton with the iterate, as after a breakdown.
#pragma once

namespace ghom {

enum { CG_RUNNING = 0, CG_CONVERGED = 1, CG_BREAKDOWN = 2, CG_CAP = 3, CG_STALLED = 4 };

constexpr int kCgStallWindow = 20;

// best: smallest r.r of the solve so far (starts at the right-hand side's b.b); since:
// iterations since it was last lowered (starts at 0).  it: iterations done, this one
// included.
constexpr int cg_status_after_iteration(double rr, double thresh, int it, int max_it, double& best, int& since) {
  if (rr <= thresh) return CG_CONVERGED;
  if (it >= max_it) return CG_CAP;
  if (rr < best) {
    best = rr;
    since = 0;
  } else {
    since += 1;
    if (since >= kCgStallWindow) return CG_STALLED;
  }
  return CG_RUNNING;
}

}  // namespace ghom
