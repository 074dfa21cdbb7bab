// Rotation gauge of full stress control (host only, no HIP).
//
// Under full stress control (every macroscopic stress component prescribed, Sec. 2.2
// eq. 19) the deformation gradient is fixed only up to the rigid rotations Q that leave
// the prescribed stress unchanged, since P(QF) = Q P(F) for an objective law: all three
// rotations at a zero stress target, the rotation about e_a for a uniaxial target
// p e_a (x) e_a.  At a stress-free state the tangent annihilates every rotation, so the
// Newton system becomes singular; under a compressive uniaxial target the rotations about
// the two transverse axes are directions of negative curvature (the dead-load instability).
//
// The gauge: when the mask prescribes all nine stress components and every row of the
// history is a multiple of e_a (x) e_a for one axis a, the three entries F_ba, F_ca, F_cb of
// the macroscopic deformation gradient, with (a, b, c) in cyclic order, are held instead of
// the matching stress components.  The history's entries there are zero, so they are held
// at their value at the start (zero from F = I).  For periodic compatible F and
// divergence-free P the average of P F^T is <P> <F>^T, and P F^T is symmetric at every
// voxel, so at equilibrium <P> <F>^T is symmetric; with the three entries of <F> at zero and
// the six other stress components at their targets this forces the three released stress
// components to their target 0.  The gauged problem therefore has the solutions of the full
// stress problem, with the rotation fixed.
#pragma once

#include <cstdint>

namespace ghom {

// axis a in 0..2 of the gauge, or -1 when it does not apply (a zero history takes a = 0)
inline int rotation_gauge_axis(const uint8_t* mask, const double* target, int nsteps) {
  for (int c = 0; c < 9; ++c)
    if (mask[c] != 1) return -1;
  for (int a = 0; a < 3; ++a) {
    bool uniaxial = true;
    for (int k = 0; k < nsteps && uniaxial; ++k)
      for (int c = 0; c < 9; ++c)
        if (c != 4 * a && target[(long long)k * 9 + c] != 0.0) {
          uniaxial = false;
          break;
        }
    if (uniaxial) return a;
  }
  return -1;
}

// components F_ba, F_ca, F_cb held by the gauge of axis a
inline void rotation_gauge_components(int a, int out[3]) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  out[0] = 3 * b + a;
  out[1] = 3 * c + a;
  out[2] = 3 * c + b;
}

// The mask the solver uses: `user` with the gauge applied when `gauge` is on and the rule
// holds.  Returns the axis (or -1).
inline int effective_mask(const uint8_t* user, const double* target, int nsteps, bool gauge, uint8_t* out) {
  for (int c = 0; c < 9; ++c) out[c] = user[c];
  if (!gauge || !target || nsteps < 1) return -1;
  const int a = rotation_gauge_axis(user, target, nsteps);
  if (a < 0) return -1;
  int comp[3];
  rotation_gauge_components(a, comp);
  for (int i = 0; i < 3; ++i) out[comp[i]] = 0;
  return a;
}

}  // namespace ghom
