"""MI355X-native generation of isogeometric systems and right-hand sides with
piece-wise constant test functions (arXiv:1910.08535).

Modules:
  iga     -- thin ctypes binding of the C ABI (include/iga.h), torch tensors in/out
  inputs  -- seeded synthetic workloads (random numbers and shapes only)
  build   -- hipcc build of libiga.so for gfx950
"""
