"""MI355X-native coupled phase-field / flow lattice Boltzmann (arXiv 2311.05097).

Submodules:
  lbmgls     ctypes binding of the C-ABI GPU library (liblbmgls.so)
  workloads  seeded synthetic inputs shared by the GPU path and the tests
"""
