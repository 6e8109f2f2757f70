"""Exact multiprecision Hankel / Toeplitz / circulant matvec on MI355X.

The compute lives in the HIP library libhmv.so (C ABI, include/hmv.h);
`paper_1402_5287_amd.hmv` is a thin ctypes binding over it that uses PyTorch
only for device memory and streams.
"""
from . import hmv  # noqa: F401
