"""MI355X-native interpolative decomposition butterfly factorization (IDBF).

The compute path is the HIP library ``libidbf.so`` built from ``csrc/`` for
gfx950; ``binding`` marshals arguments to its C ABI (``include/idbf.h``).
Importing this package loads nothing; the library is loaded on first use
and its absence is an error, never a fallback.
"""
__all__ = ["inputs", "binding"]
