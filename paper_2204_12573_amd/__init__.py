"""MI355X-native evaluation of the FLARE B2 Bayesian force field (energies, forces,
per-atom uncertainty), with hand-written HIP kernels for gfx950 behind a C ABI.

Submodules:
  structures  seeded synthetic inputs (no force-field arithmetic)
  binding     ctypes binding of the C ABI (libflare_mi355x.so)
  engine      device-resident state, MD driver
"""
