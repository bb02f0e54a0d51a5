"""MI355X-native Monte Carlo dose engine for the analytic phase-space-ring
linac source model (Tian et al., arXiv:1503.01725).

Submodules:
  workloads -- seeded synthetic inputs (models, phantoms, beams)
  _native   -- ctypes binding of libpsl.so (include/psl.h)
  engine    -- Python objects over the binding (torch for device memory)
  build     -- compiles libpsl.so for gfx950
"""
__all__ = ["workloads", "engine", "build"]
