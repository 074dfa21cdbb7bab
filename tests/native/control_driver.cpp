// Prints the effective control mask and the rotation-gauge axis (csrc/control.hpp) for a
// mask and a history given on the command line (host only; built by the tests with g++).
// argv: gauge(0/1) m0..m8 nsteps t[0][0..8] t[1][0..8] ...   output: "axis m0 .. m8"
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1901_06531_amd/csrc/control.hpp"

int main(int argc, char** argv) {
  if (argc < 12) return 2;
  const bool gauge = std::atoi(argv[1]) != 0;
  uint8_t user[9], out[9];
  for (int c = 0; c < 9; ++c) user[c] = (uint8_t)std::atoi(argv[2 + c]);
  const int nsteps = std::atoi(argv[11]);
  if (argc != 12 + 9 * nsteps) return 2;
  std::vector<double> t(9 * (size_t)nsteps);
  for (size_t i = 0; i < t.size(); ++i) t[i] = std::atof(argv[12 + i]);
  const int axis = ghom::effective_mask(user, nsteps ? t.data() : nullptr, nsteps, gauge, out);
  std::printf("%d", axis);
  for (int c = 0; c < 9; ++c) std::printf(" %d", (int)out[c]);
  std::printf("\n");
  return 0;
}
