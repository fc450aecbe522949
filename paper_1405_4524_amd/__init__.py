"""MI355X-native stochastic all-to-all propagators (Giedt & Howarth, arXiv:1405.4524).

The compute path is the HIP library ``liba2a.so`` (sources in ``csrc/``, C ABI in
``include/a2a.h``); ``a2a`` is its thin ctypes binding and ``inputs`` draws the seeded
synthetic gauge fields and noise sources.  Import ``paper_1405_4524_amd.a2a`` for the
library; this package module itself loads nothing.
"""
__all__ = ["a2a", "inputs"]
