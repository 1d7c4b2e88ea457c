"""MI355X (gfx950) implementation of one SSP-RK3 stage of the
positivity-preserving Active Flux scheme for 2D ideal MHD with the
Godunov-Powell source term (arXiv 2506.04857).

Modules:
  af_mhd   thin ctypes binding of the HIP library libaf_mhd.so (C ABI in include/af_mhd.h)
  inputs   seeded synthetic problem set-ups and initial data
  build    hipcc build of the library
"""
