"""MI355X-native Chebyshev-filtered subspace iteration (CheFSI) for real-space Kohn-Sham DFT.

The compute path lives in the HIP library ``libchefsi.so`` (sources in ``csrc/``,
C-ABI in ``include/chefsi.h``); ``chefsi`` holds the ctypes binding and
``inputs`` the seeded synthetic problem generator.  Importing this package
loads nothing: import ``paper_2302_09708_amd.chefsi`` to load the library.
"""
