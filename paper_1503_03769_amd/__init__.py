"""MI355X (gfx950) implementation of the per-step recursion of the distributed
computation particle PHD filter (arXiv 1503.03769).

Modules:
  pphd      -- ctypes binding of libpphd (the C ABI in include/pphd.h)
  scenario  -- seeded synthetic inputs (truth tracks, measurement sets)
  metrics   -- OSPA miss distance used by the benchmark
  build     -- hipcc build of libpphd.so
"""
