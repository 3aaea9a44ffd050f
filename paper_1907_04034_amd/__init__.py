"""MI355X-native EDAC-SPH wind-tunnel hot path (arXiv 1907.04034).

Submodules:
  inputs   -- seeded synthetic particle sets and workload parameters
  binding  -- ctypes binding of libsph.so (the HIP path); loads lazily
  build    -- compiles libsph.so for gfx950 with hipcc
"""
