"""MI355X-native RNS-CKKS homomorphic matrix product (arXiv 2305.17341).

The compute lives in a HIP/C++ shared library with a C ABI
(include/he_mi355x.h); ``paper_2305_17341_amd.he`` is the thin ctypes binding.
Importing the package does not load the library.
"""
__all__ = ["he", "inputs"]
