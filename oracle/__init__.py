"""CPU oracle for the force-approach pseudopotential LBM (arXiv:2003.07968).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library (the HIP path)
never imports it, and it imports nothing from the product library.

  lbmref     ctypes binding of the plain FP64 C oracle (lbmref.c)
  analytics  the macroscopic theory of Sec. II.B and IV (coexistence, planar
             surface tension, Lamb period), in NumPy/SciPy FP64
"""
