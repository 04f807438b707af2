"""MI355X-native rejection-ABC hot path for the stochastic COVID-19
compartment model of arXiv 2012.14332.

The compute runs in hand-written HIP kernels behind the C ABI of
``include/abc.h`` (``libabc.so``); ``paper_2012_14332_amd.abc`` is the thin
ctypes binding. Importing the package does not load the library; the first
call does, and fails loudly if it is missing.
"""
