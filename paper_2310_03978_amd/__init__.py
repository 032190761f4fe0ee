"""Sliced tensor-network contraction of random quantum circuits on MI355X (gfx950).

The compute path is the HIP library built from ``csrc/`` (C ABI in
``include/tn.h``); ``tn`` is its ctypes binding.
"""
