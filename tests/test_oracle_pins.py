"""Pins of the CPU oracle against things other than itself (CPU only).

* the brute-force state vector (which never builds a tensor network);
* hand-derived closed forms (tests/golden/closed_forms.txt);
* normalisation of the full output state;
* slicing invariance and the slice-id convention;
* path invariance;
* explicit-loop contraction of small random networks with batch, trace and
  hyperedge labels and extents 1, 2, 4;
* the dense-matrix state vector (pins the state-vector simulator itself);
* Porter-Thomas moments of deep random circuits.
"""
import os

import numpy as np
import pytest

from oracle import contract, metrics, naive, statevector
from tn_inputs import configs
from tn_inputs.circuits import (SINGLE_QUBIT_GATES, Circuit, Gate, fsim, open_and_closed,
                                product_circuit, random_circuit)
from tn_inputs.network import Network, circuit_network, random_network
from tn_inputs.paths import choose_slices, find_path, greedy_path

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, vals = line.split("|")
        amps = []
        for pair in vals.split(";"):
            re, im = pair.split(",")
            amps.append(complex(float(re), float(im)))
        out[name.strip()] = np.array(amps)
    return out


def _oracle(net, path=None, sliced=(), slice_ids=None):
    if path is None:
        path = greedy_path(net.labels, net.open_labels, net.extents(), seed=0)
    return contract.amplitudes(net.tensors, net.labels, net.open_labels, path, sliced, slice_ids)


def _sv(circ, open_q, closed):
    psi = statevector.simulate(circ)
    return statevector.subspace_amplitudes(psi, open_q, closed)


def test_rqc12_matches_state_vector():
    circ, net, best = configs.build("rqc12")
    a = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    ref = _sv(circ, net.meta["open_qubits"], net.meta["closed_bits"])
    assert a.shape == (16,)
    assert metrics.rel_l2(a, ref) <= 1e-12


@pytest.mark.parametrize("rows,cols,cycles,k,seed", [(2, 3, 6, 3, 7), (3, 3, 10, 2, 8),
                                                     (4, 4, 8, 5, 9), (3, 5, 6, 0, 10)])
def test_random_circuits_match_state_vector(rows, cols, cycles, k, seed):
    circ = random_circuit(rows, cols, cycles, seed)
    open_q, closed = open_and_closed(circ.n_qubits, k, seed + 1)
    net = circuit_network(circ, open_q, closed)
    a = _oracle(net)
    ref = _sv(circ, open_q, closed)
    assert metrics.rel_l2(a, ref) <= 1e-12


def test_full_state_norm_is_one():
    circ = random_circuit(3, 4, 8, 101)
    net = circuit_network(circ, tuple(range(12)), {})
    a = _oracle(net)
    assert a.shape == (4096,)
    assert abs(np.vdot(a, a).real - 1.0) <= 1e-12


def test_closed_forms():
    g = _golden()
    for name in ("sqrt_x", "sqrt_y", "sqrt_w"):
        circ = product_circuit(1, [name])
        net = circuit_network(circ, (0,), {})
        np.testing.assert_allclose(_oracle(net), g[f"{name}_on_0"], atol=1e-15)
    # fSim on a prepared basis state: hand-built network ket(x0) ket(x1) -> fSim -> open
    for bits, key in (((0, 1), "fsim_pi6_pi5_on_01"), ((1, 1), "fsim_pi6_pi5_on_11")):
        kets = [np.eye(2, dtype=np.complex128)[b] for b in bits]
        gate = fsim(np.pi / 6, np.pi / 5).reshape(2, 2, 2, 2)
        net = Network(tensors=kets + [gate], labels=[(0,), (1,), (2, 3, 0, 1)],
                      open_labels=(2, 3))
        np.testing.assert_allclose(_oracle(net), g[key], atol=1e-15)


def test_empty_circuit_and_product_states():
    circ = Circuit(n_qubits=3, sites=[(0, 0), (0, 1), (0, 2)])
    net = circuit_network(circ, (1,), {0: 0, 2: 0})
    np.testing.assert_allclose(_oracle(net), [1.0, 0.0], atol=1e-15)
    names = ["sqrt_x", "sqrt_w", "sqrt_y", "sqrt_x"]
    circ = product_circuit(4, names)
    net = circuit_network(circ, (0, 1, 2, 3), {})
    col = [SINGLE_QUBIT_GATES[n][:, 0] for n in names]
    expect = col[0]
    for c in col[1:]:
        expect = np.kron(expect, c)
    np.testing.assert_allclose(_oracle(net), expect, atol=1e-15)


def test_slicing_invariance():
    circ, net, best = configs.build("rqc12")
    ext = net.extents()
    full = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    sliced = choose_slices(net.labels, net.open_labels, ext, best["path"], cap_log2=6,
                           min_sliced=3)
    assert len(sliced) >= 3
    parts = [contract.contract_slice(net.tensors, net.labels, net.open_labels, best["path"],
                                     sliced, s) for s in range(2 ** len(sliced))]
    total = np.sum(parts, axis=0)
    assert np.max(np.abs(total - full)) <= 1e-13
    # the slices are genuinely different sub-tasks
    assert np.max(np.abs(parts[0] - parts[1])) > 1e-6


def test_slice_id_convention():
    """Slice s fixes the first sliced label to its most significant digit."""
    net = random_network(5, n_tensors=5, n_labels=8, extents=(2, 4), n_open=1,
                         allow_hyper=False, allow_trace=False)
    ext = net.extents()
    cands = [l for l in ext if l not in net.open_labels and ext[l] > 1]
    sliced = cands[:2]
    path = greedy_path(net.labels, net.open_labels, ext, seed=1)
    e0, e1 = ext[sliced[0]], ext[sliced[1]]
    for s in range(e0 * e1):
        v0, v1 = s // e1, s % e1
        proj = [np.eye(e0, dtype=np.complex128)[v0], np.eye(e1, dtype=np.complex128)[v1]]
        ref = naive.amplitudes(net.tensors + proj, net.labels + [(sliced[0],), (sliced[1],)],
                               net.open_labels)
        got = contract.contract_slice(net.tensors, net.labels, net.open_labels, path, sliced, s)
        np.testing.assert_allclose(got, ref, atol=1e-11)


def test_path_invariance():
    circ, net, best = configs.build("rqc12")
    a = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    for seed in (3, 4):
        p = greedy_path(net.labels, net.open_labels, net.extents(), seed=seed, temperature=0.05)
        assert p != best["path"]
        b = contract.amplitudes(net.tensors, net.labels, net.open_labels, p)
        assert np.max(np.abs(a - b)) <= 1e-13


@pytest.mark.parametrize("seed", range(8))
def test_pairwise_matches_explicit_loops(seed):
    net = random_network(seed, n_tensors=5, n_labels=8, extents=(1, 2, 3), n_open=2)
    path = greedy_path(net.labels, net.open_labels, _pow2_ok(net), seed=seed) \
        if _pow2(net) else _any_path(net)
    a = contract.amplitudes(net.tensors, net.labels, net.open_labels, path)
    ref = naive.amplitudes(net.tensors, net.labels, net.open_labels)
    np.testing.assert_allclose(a, ref, rtol=1e-12, atol=1e-12)


def _pow2(net):
    return all((e & (e - 1)) == 0 for e in net.extents().values())


def _pow2_ok(net):
    return net.extents()


def _any_path(net):
    # linear path: fold every tensor into slot 0 in order
    return [(0, j) for j in range(1, len(net.tensors))]


def test_batch_labels_are_carried():
    """A hyperedge shared by both operands and a third tensor is carried, not summed."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    B = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    C = rng.standard_normal((2,)) + 1j * rng.standard_normal((2,))
    labels = [(0, 1), (0, 1), (0,)]
    a = contract.amplitudes([A, B, C], labels, (), [(0, 1), (0, 2)])
    ref = np.sum(C * np.sum(A * B, axis=1))
    assert abs(a[0] - ref) <= 1e-12


def test_dense_statevector_pins_gate_application():
    for seed in (1, 2):
        circ = random_circuit(2, 3, 5, seed)
        psi = statevector.simulate(circ).reshape(-1)
        dense = statevector.full_unitary_apply(circ)
        np.testing.assert_allclose(psi, dense, atol=1e-13)


def test_gates_are_unitary():
    for u in list(SINGLE_QUBIT_GATES.values()) + [fsim(0.3, 0.7)]:
        np.testing.assert_allclose(u @ u.conj().T, np.eye(u.shape[0]), atol=1e-15)


def test_porter_thomas_moments():
    circ = random_circuit(4, 4, 32, 17)
    psi = statevector.simulate(circ).reshape(-1)
    p = np.abs(psi) ** 2 * psi.size
    assert abs(p.mean() - 1.0) <= 1e-12
    assert abs(np.mean(p ** 2) - 2.0) <= 0.1


def test_metrics_closed_forms():
    ref = np.array([1.0, 1j, -1.0, 0.5])
    assert metrics.rel_l2(ref, ref) == 0.0
    assert abs(metrics.eps_l2sq(2 * ref, ref) - 3.0) <= 1e-15
    assert abs(metrics.fidelity(1j * ref, ref) - 1.0) <= 1e-15
    uniform = np.full(8, 2 ** -2.5)  # 5 qubits, p = 2^-5 for each of 8 strings
    assert abs(metrics.lxeb(uniform, 5)) <= 1e-15


def test_step_costs_closed_form():
    """flops = 8*B*M*N*K and bytes = 8(|A|+|B|+|C|) on a hand-sized example."""
    A = np.zeros((2, 4, 8))   # labels (0 batch, 1 summed, 2 free)
    B = np.zeros((2, 4, 2))   # labels (0 batch, 1 summed, 3 free)
    C = np.zeros((2,))        # label 0 keeps the batch label alive
    costs = contract.step_costs([A, B, C], [(0, 1, 2), (0, 1, 3), (0,)], (2, 3),
                                [(0, 1), (0, 2)])
    s = costs[0]
    assert (s["B"], s["M"], s["N"], s["K"]) == (2, 8, 2, 4)
    assert s["flops"] == 8 * 2 * 8 * 2 * 4
    assert s["bytes"] == 8 * (64 + 16 + 32)
