"""Seeded vectors for the dot-product precision study (input generator only).

The extended-precision study of Sec. 4.2 multiplies vectors whose entries have
random signs and magnitudes spread over ten decades, from 1e-7 to 1e3 (the
range the paper calls the FP16 range).  Magnitudes are drawn log-uniformly over
that range, signs uniformly; numpy's PCG64 generator (``default_rng``).  The
values are rounded to float32 here, because both the GPU path and the oracle
take float32 operands.  No arithmetic of the method lives here.
"""
from __future__ import annotations

import numpy as np

FP16_RANGE = (1e-7, 1e3)


def log_uniform_pairs(count: int, length: int, seed: int, lo: float = FP16_RANGE[0],
                      hi: float = FP16_RANGE[1]):
    """(a, b): two float32 arrays of shape (count, length), |entries| log-uniform in
    [lo, hi] with random signs."""
    rng = np.random.default_rng(seed)

    def draw():
        mag = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(count, length)))
        sign = np.where(rng.integers(0, 2, size=(count, length)) == 1, 1.0, -1.0)
        return (sign * mag).astype(np.float32)

    return draw(), draw()
