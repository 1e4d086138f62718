"""MI355X-native homomorphic linear layers of CryptoTrain (arXiv 2409.16675).

The compute path lives in ``libhe.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/he.h``); ``he`` is a thin ctypes binding with the same
names.  PyTorch is used only for device memory and streams.
"""
