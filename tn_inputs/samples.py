"""Synthetic bitstring samples standing in for an experiment's (input generator only).

The paper verifies samples taken on a quantum device (Sec. 2.2, Sec. 5); they are not
available here.  A device of fidelity F is modelled as the mixture F p + (1 - F) uniform
over the 2^N bitstrings (F = 1: ideal samples, F = 0: pure noise), for which the LXEB
estimator's expectation is F times that of ideal samples.  Draws use numpy's PCG64
generator; the probabilities p come from the caller (any exact simulation).
"""
from __future__ import annotations

import numpy as np


def sample_with_fidelity(probs, count: int, fidelity: float, seed: int) -> np.ndarray:
    """Indices of `count` bitstrings: each drawn from probs (normalised here) with
    probability `fidelity`, else uniformly."""
    p = np.asarray(probs, dtype=np.float64)
    p = p / p.sum()
    rng = np.random.default_rng(seed)
    ideal = rng.random(count) < fidelity
    out = rng.integers(0, p.size, size=count)
    out[ideal] = rng.choice(p.size, size=int(ideal.sum()), p=p)
    return out


def index_to_bits(idx, n_qubits: int) -> np.ndarray:
    """uint8 rows of the bitstrings with the given state indices (qubit 0 most significant)."""
    idx = np.asarray(idx, dtype=np.int64)
    shifts = np.arange(n_qubits - 1, -1, -1, dtype=np.int64)
    return ((idx[:, None] >> shifts[None, :]) & 1).astype(np.uint8)
