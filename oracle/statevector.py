"""Brute-force state-vector simulation (independent check of the contraction oracle).

TEST INFRASTRUCTURE ONLY.  Starts from |0...0> and applies every gate in
circuit order to a (2,)*n complex128 array; qubit 0 is the most significant bit
of the state index.  It never builds a tensor network, so it pins the
circuit-to-network mapping and the contraction together.
"""
from __future__ import annotations

import numpy as np


def apply_gate(psi: np.ndarray, matrix: np.ndarray, qubits) -> np.ndarray:
    k = len(qubits)
    g = np.asarray(matrix, dtype=np.complex128).reshape((2,) * (2 * k))
    out = np.tensordot(g, psi, axes=(list(range(k, 2 * k)), list(qubits)))
    return np.moveaxis(out, list(range(k)), list(qubits))


def simulate(circ) -> np.ndarray:
    n = circ.n_qubits
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for g in circ.gates:
        psi = apply_gate(psi, g.matrix, g.qubits)
    return psi


def subspace_amplitudes(psi: np.ndarray, open_qubits, closed_bits: dict) -> np.ndarray:
    """Amplitudes over the open qubits (first open qubit most significant)."""
    n = psi.ndim
    index = []
    for q in range(n):
        index.append(slice(None) if q in open_qubits else closed_bits[q])
    sub = psi[tuple(index)]
    return np.ascontiguousarray(sub).reshape(-1)


def full_unitary_apply(circ) -> np.ndarray:
    """Same state built from dense 2^n x 2^n gate matrices (n <= 8): pins apply_gate."""
    n = circ.n_qubits
    dim = 2 ** n
    state = np.zeros(dim, dtype=np.complex128)
    state[0] = 1.0
    for g in circ.gates:
        full = _embed(g.matrix, g.qubits, n)
        state = full @ state
    return state


def _embed(matrix, qubits, n):
    dim = 2 ** n
    k = len(qubits)
    full = np.zeros((dim, dim), dtype=np.complex128)
    for col in range(dim):
        bits = [(col >> (n - 1 - q)) & 1 for q in range(n)]
        sub_in = 0
        for q in qubits:
            sub_in = 2 * sub_in + bits[q]
        for sub_out in range(2 ** k):
            amp = matrix[sub_out, sub_in]
            if amp == 0:
                continue
            nb = list(bits)
            for p, q in enumerate(qubits):
                nb[q] = (sub_out >> (k - 1 - p)) & 1
            row = 0
            for b in nb:
                row = 2 * row + b
            full[row, col] += amp
    return full
