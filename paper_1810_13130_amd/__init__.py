"""MI355X-native hot path of real-time TDDFT with spectral finite elements.

The compute lives in the HIP library ``libtdfe.so`` (C ABI in
``include/tdfe.h``); ``tdfe`` is its ctypes binding.
"""
from . import tdfe  # noqa: F401
