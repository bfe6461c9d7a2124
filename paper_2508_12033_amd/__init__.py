"""MI355X-native lattice-regularized diffusion Monte Carlo hot path.

Submodules:
  inputs  -- seeded synthetic molecular systems (no method arithmetic)
  lrdmc   -- ctypes binding of the HIP library liblrdmc.so (C ABI: include/lrdmc.h)
  build   -- hipcc build of liblrdmc.so for gfx950
"""
