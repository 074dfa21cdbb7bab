// Drives the adaptive-stepping controller with a scripted sequence of sub-increment
// outcomes and prints its state after each event (host only; built by the tests with g++).
// argv: max_cuts grow_below start_fraction outcome...   outcome: "f" (failed) or a Newton
// iteration count (converged).
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../paper_1901_06531_amd/csrc/substep.hpp"

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  ghom::SubstepClock clk(std::atoi(argv[1]), std::atoi(argv[2]), std::atof(argv[3]));
  std::printf("start %.17g %.17g %d\n", clk.theta, clk.dtheta, (int)clk.done());
  for (int i = 4; i < argc && !clk.done(); ++i) {
    const double end = clk.next_end();
    if (std::strcmp(argv[i], "f") == 0) {
      const bool ok = clk.reject();
      std::printf("reject %.17g %.17g %.17g %d %d\n", end, clk.theta, clk.dtheta, clk.cuts, (int)ok);
      if (!ok) return 0;
    } else {
      clk.accept(std::atoi(argv[i]));
      std::printf("accept %.17g %.17g %.17g %d\n", end, clk.theta, clk.dtheta, (int)clk.done());
    }
  }
  double a[9], b[9], m[9];
  for (int i = 0; i < 9; ++i) {
    a[i] = 0.1 * i + 0.3;
    b[i] = 1.0 / (i + 3.0);
  }
  ghom::lerp9(a, b, 1.0, m);
  int exact = 1;
  for (int i = 0; i < 9; ++i) exact = exact && m[i] == b[i];
  ghom::lerp9(a, b, 0.25, m);
  std::printf("lerp %d %.17g\n", exact, m[4]);
  return 0;
}
