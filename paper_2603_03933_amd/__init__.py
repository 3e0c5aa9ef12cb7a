"""MI355X-native IMEX trust-region hot path for the Landau-Brazovskii energy.

The compute path is the HIP library ``liblbtr.so`` behind the C ABI declared in
``include/lb.h``; ``paper_2603_03933_amd.lb`` is a thin ctypes binding to it.
Importing the package does not load the library: the first call does, and it
raises if the library is missing.
"""
