"""MI355X-native Galerkin-FFT homogenization with stress / mixed control.

Submodules:
  ghom   -- ctypes binding of the C-ABI library libghom.so (HIP kernels for gfx950)
  synth  -- seeded synthetic microstructures, material tables and load histories
  build  -- compiles libghom.so with hipcc

Importing the package loads nothing native; ``paper_1901_06531_amd.ghom`` does.
"""
