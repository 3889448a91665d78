"""MI355X-native Penning-trap ion-crystal simulator (FMM Coulomb forces).

The compute path lives in the HIP shared library built from ``csrc/``; the
Python side (``native``) only marshals arguments through its C ABI.  Importing
this package does not load the library; ``native.load()`` does, and fails
loudly when it is missing.
"""
__all__ = ["inputs", "native"]
