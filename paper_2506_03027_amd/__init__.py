"""MI355X-native asynchrony-tolerant compressible-flow solver (arXiv 2506.03027).

The solver lives in the HIP library ``libatns.so`` (C ABI in include/atns.h);
``atns`` is its ctypes binding and ``inputs`` generates the synthetic inputs.
"""
