"""Circuit -> tensor network mapping and random test networks (input generator).

Sec. 2.1 of the paper maps each gate to a tensor and each wire segment to a
bond; the network is closed on the initial-state side and open on the
final-state side.  Appendix A.1 describes the subspace variant used here:
closed qubits get a projector onto a fixed bit at the output, open qubits keep
their output bond, so contracting the network yields the 2^k "correlated"
amplitudes of the open qubits.

Conventions (fixed here, shared by every consumer of these inputs):

* every tensor is complex128, row-major in its label order, extent 2 per label;
* a one-qubit gate U has labels (out, in) and data U[out, in];
* a two-qubit gate G on (a, b) has labels (a_out, b_out, a_in, b_in) and data
  G.reshape(2, 2, 2, 2) (basis index 2*x_a + x_b);
* the initial state |0> of a qubit is the vector [1, 0]; the output projector
  onto bit x is the unit vector e_x;
* open labels are listed in increasing qubit order, the first one being the
  most significant bit of the amplitude index.

No contraction is done here: every leaf is a single gate, ket or bra.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Network:
    tensors: list          # list[np.ndarray], complex128
    labels: list           # list[tuple[int, ...]]
    open_labels: tuple     # output order, first = most significant
    n_labels: int = 0
    meta: dict = None

    def extents(self) -> dict:
        ext = {}
        for t, lab in zip(self.tensors, self.labels):
            for l, e in zip(lab, t.shape):
                ext[l] = int(e)
        return ext


def circuit_network(circ, open_qubits, closed_bits: dict) -> Network:
    """Tensor network of <x_closed| U |0...0> with the open qubits' outputs left open."""
    n = circ.n_qubits
    next_label = 0
    wire = [0] * n
    tensors, labels = [], []

    def fresh():
        nonlocal next_label
        next_label += 1
        return next_label - 1

    ket = np.array([1.0, 0.0], dtype=np.complex128)
    for q in range(n):
        wire[q] = fresh()
        tensors.append(ket.copy())
        labels.append((wire[q],))
    for g in circ.gates:
        if len(g.qubits) == 1:
            (q,) = g.qubits
            new = fresh()
            tensors.append(np.array(g.matrix, dtype=np.complex128))
            labels.append((new, wire[q]))
            wire[q] = new
        else:
            qa, qb = g.qubits
            na, nb = fresh(), fresh()
            tensors.append(np.array(g.matrix, dtype=np.complex128).reshape(2, 2, 2, 2))
            labels.append((na, nb, wire[qa], wire[qb]))
            wire[qa], wire[qb] = na, nb
    open_set = set(open_qubits)
    for q in range(n):
        if q in open_set:
            continue
        bra = np.zeros(2, dtype=np.complex128)
        bra[closed_bits[q]] = 1.0
        tensors.append(bra)
        labels.append((wire[q],))
    open_labels = tuple(wire[q] for q in sorted(open_set))
    return Network(tensors=tensors, labels=labels, open_labels=open_labels,
                   n_labels=next_label,
                   meta={"n_qubits": n, "open_qubits": tuple(sorted(open_set)),
                         "closed_bits": dict(closed_bits)})


def random_network(seed: int, n_tensors: int = 6, n_labels: int = 9, max_rank: int = 4,
                   extents=(1, 2, 4), n_open: int = 2, allow_hyper: bool = True,
                   allow_trace: bool = True) -> Network:
    """Small random network for fuzzing label handling.

    Labels may appear in one tensor (a summed "trace" label unless open), two
    tensors (an ordinary bond) or, with ``allow_hyper``, three tensors (a
    hyperedge, which becomes a batch label when two of its tensors meet).
    Every tensor is connected to the others so that a pairwise path exists.
    Values are complex normal.
    """
    rng = np.random.default_rng(seed)
    ext = {l: int(rng.choice(extents)) for l in range(n_labels)}
    occ = {l: [] for l in range(n_labels)}
    tensor_labels = [[] for _ in range(n_tensors)]
    # spanning chain keeps the network connected
    order = rng.permutation(n_tensors)
    l = 0
    for a, b in zip(order[:-1], order[1:]):
        tensor_labels[a].append(l); tensor_labels[b].append(l)
        l += 1
    while l < n_labels:
        kind = rng.integers(0, 3)
        if kind == 0 and allow_trace:
            cnt = 1
        elif kind == 2 and allow_hyper and n_tensors >= 3:
            cnt = 3
        else:
            cnt = 2
        ts = rng.choice(n_tensors, size=cnt, replace=False)
        for t in ts:
            if len(tensor_labels[t]) < max_rank:
                tensor_labels[t].append(l)
        l += 1
    for t in range(n_tensors):
        for lab in tensor_labels[t]:
            occ[lab].append(t)
    used = [lab for lab in range(n_labels) if occ[lab]]
    open_candidates = list(used)
    rng.shuffle(open_candidates)
    open_labels = tuple(open_candidates[:n_open])
    tensors, labels = [], []
    for t in range(n_tensors):
        lab = tuple(int(x) for x in rng.permutation(tensor_labels[t]))
        shape = tuple(ext[x] for x in lab)
        data = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        tensors.append(np.asarray(data, dtype=np.complex128))
        labels.append(lab)
    return Network(tensors=tensors, labels=labels, open_labels=open_labels,
                   n_labels=n_labels, meta={"seed": seed})
