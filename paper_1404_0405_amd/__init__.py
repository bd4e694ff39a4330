"""MI355X-native adaptive wavelet TRiSK shallow-water library (arXiv:1404.0405).

The compute path is the HIP library ``libwt.so`` (C ABI in ``include/wt.h``); ``wt`` is its
ctypes binding and ``inputs`` the seeded initial-condition generators.
"""
