"""Pins of the sparse-state oracle (oracle/sparse.py) against things other than itself:
the paper's worked example of the sparse einsum (Sec. 3.3), the per-bitstring definition,
the dense all-open contraction read at the bitstrings, and slicing invariance."""
import os

import numpy as np
import pytest

from oracle import contract, sparse
from tn_inputs import configs
from tn_inputs.circuits import open_and_closed, random_circuit, sample_bitstrings
from tn_inputs.network import circuit_network
from tn_inputs.paths import choose_slices, greedy_path

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sparse_einsum_example.txt")


def _read_example():
    rows, sections = [], []
    for line in open(GOLDEN):
        if line.startswith("# bitstrings"):
            sections.append([])
        elif line.startswith("# merged"):
            sections.append([])
        elif line.strip() and not line.startswith("#"):
            sections[-1].append([int(c) for c in line.strip()])
    return np.array(sections[0], dtype=np.uint8), np.array(sections[1], dtype=np.uint8)


def test_worked_example_of_the_sparse_einsum():
    bits, merged = _read_example()
    rng = np.random.default_rng(3)
    # labels: a=0, b=1, c=2 (open), d=3, e=4 (open), q0's bond = 5 (open, on its own leaf)
    F = rng.standard_normal((2, 2, 2, 3)) + 1j * rng.standard_normal((2, 2, 2, 3))   # F[c, a, b, d]
    H = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))               # H[e, d]
    keys_all = sparse.bit_keys(bits[:, 1:])                                          # columns (c, e)
    A = sparse._merged_leaf(F, (2, 0, 1, 3), {2: 0, 4: 1}, keys_all)
    B = sparse._merged_leaf(H, (4, 3), {2: 0, 4: 1}, keys_all)
    L, lab, mask, keys = sparse._step(A, B, {0, 1}, keys_all)
    assert len(keys) == len(merged) == 2
    assert [[int(k) & 1, (int(k) >> 1) & 1] for k in keys] == merged.tolist()
    assert lab == (0, 1)
    for f, (c, e) in enumerate(merged):
        want = np.tensordot(F[c], H[e], axes=([2], [0]))      # sum_d F[c, a, b, d] H[e, d]
        np.testing.assert_allclose(L[f], want, rtol=1e-14, atol=1e-14)


def _all_open(rows, cols, cycles, seed):
    circ = random_circuit(rows, cols, cycles, seed)
    oq, _ = open_and_closed(circ.n_qubits, circ.n_qubits, seed)
    net = circuit_network(circ, oq, {})
    path = greedy_path(net.labels, net.open_labels, net.extents(), seed=seed)
    return circ, net, path


@pytest.mark.parametrize("seed", [0, 1])
def test_sparse_state_matches_definition_and_dense(seed):
    circ, net, path = _all_open(3, 3, 6, 700 + seed)
    bits = sample_bitstrings(circ.n_qubits, 40, seed, duplicates=6)
    got = sparse.sparse_state_amplitudes(net.tensors, net.labels, net.open_labels, path, bits)
    ref = sparse.definition_amplitudes(net.tensors, net.labels, net.open_labels, path, bits)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15)
    dense = contract.amplitudes(net.tensors, net.labels, net.open_labels, path)
    idx = [int("".join(str(int(b)) for b in row), 2) for row in bits]   # first open label most significant
    np.testing.assert_allclose(got, dense[idx], rtol=1e-12, atol=1e-15)


def test_sparse_state_single_bitstring_and_every_bitstring():
    circ, net, path = _all_open(2, 3, 5, 711)
    n = circ.n_qubits
    every = np.array([[(v >> (n - 1 - i)) & 1 for i in range(n)] for v in range(1 << n)], dtype=np.uint8)
    got = sparse.sparse_state_amplitudes(net.tensors, net.labels, net.open_labels, path, every)
    dense = contract.amplitudes(net.tensors, net.labels, net.open_labels, path)
    np.testing.assert_allclose(got, dense, rtol=1e-12, atol=1e-15)
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) <= 1e-12                  # the full state is normalised
    one = sparse.sparse_state_amplitudes(net.tensors, net.labels, net.open_labels, path, every[5:6])
    np.testing.assert_allclose(one, dense[5:6], rtol=1e-12, atol=1e-15)


def test_sparse_state_slicing_invariance():
    circ, net, path = _all_open(3, 3, 6, 720)
    bits = sample_bitstrings(circ.n_qubits, 30, 4)
    sliced = choose_slices(net.labels, net.open_labels, net.extents(), path, cap_log2=6, min_sliced=3,
                           max_sliced=3)
    whole = sparse.sparse_state_amplitudes(net.tensors, net.labels, net.open_labels, path, bits)
    parts = sparse.sparse_state_amplitudes(net.tensors, net.labels, net.open_labels, path, bits, sliced)
    np.testing.assert_allclose(parts, whole, rtol=1e-12, atol=1e-15)
