"""MI355X-native D2Q9 force-approach pseudopotential lattice Boltzmann update
(arXiv:2003.07968).

  paper_2003_07968_amd.lbm        ctypes binding of the C-ABI library liblbm.so
                                  (HIP kernels for gfx950); imported on demand
  paper_2003_07968_amd.workloads  seeded synthetic initial states and parameters
"""
