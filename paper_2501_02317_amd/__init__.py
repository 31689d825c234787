"""MI355X-native Godunov hydrodynamics hot path (arXiv 2501.02317, Sec. 3).

Submodules:
  hydro      -- ctypes binding of the HIP library libhydro.so (C ABI in
                include/hydro.h).  Importing it loads the library and fails
                loudly if it has not been built.
  workloads  -- seeded synthetic initial conditions (primitive fields only).
  build      -- compiles the HIP library for gfx950.
"""
