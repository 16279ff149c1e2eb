"""MI355X-native pseudospectral Navier-Stokes / MHD hot path.

Submodules:
  inputs  seeded synthetic initial fields and forcing (no method arithmetic)
  pst     ctypes binding over the C ABI of the HIP library (libpst.so)
  build   compiles the HIP library for gfx950

Importing the package loads nothing; ``paper_1808_01309_amd.pst`` loads the
HIP library and raises if it is missing.
"""
