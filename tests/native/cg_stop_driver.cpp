// Drives the CG stopping rule (csrc/cg_stop.hpp) with a scripted sequence of r.r values and
// prints the status after each iteration (host only; built by the tests with g++).
// argv: rr0 thresh max_it rr_1 rr_2 ...   output: one line "it status best since" per value,
// ending at the first non-running status.
#include <cstdio>
#include <cstdlib>

#include "../../paper_1901_06531_amd/csrc/cg_stop.hpp"

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  double best = std::atof(argv[1]);
  const double thresh = std::atof(argv[2]);
  const int max_it = std::atoi(argv[3]);
  int since = 0;
  std::printf("window %d\n", ghom::kCgStallWindow);
  for (int i = 4, it = 1; i < argc; ++i, ++it) {
    const int st = ghom::cg_status_after_iteration(std::atof(argv[i]), thresh, it, max_it, best, since);
    std::printf("%d %d %.17g %d\n", it, st, best, since);
    if (st != ghom::CG_RUNNING) break;
  }
  return 0;
}
