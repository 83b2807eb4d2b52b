"""MI355X-native fused stream-collide step of the non-ideal compressible
double-distribution lattice Boltzmann method (arXiv 2510.14712).

The compute path is the HIP library ``liblbm_hip.so`` behind the C ABI
declared in ``include/lbm.h``; ``paper_2510_14712_amd.lbm`` is its thin
ctypes binding.  ``inputs`` holds the seeded synthetic initial conditions.
"""
