"""The benchmark and test workloads, with their seeds (synthetic stand-ins).

The paper's workloads are Sycamore circuits with experimental bitstrings,
which are not available; seeded lattice circuits of the same gate family stand
in for them.  Each workload fixes the lattice, depth, number of open qubits
(correlated amplitudes of the last k qubits), the closed-bit seed, the memory
cap (log2 elements of the largest intermediate) and the number of sliced bonds.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

from .circuits import open_and_closed, random_circuit
from .network import circuit_network
from .paths import find_path


@dataclass(frozen=True)
class Workload:
    name: str
    rows: int
    cols: int
    cycles: int
    k_open: int
    circuit_seed: int
    closed_seed: int
    cap_log2: int
    n_sliced: int = 0
    removed: tuple = ()
    trials: int = 8
    description: str = ""


WORKLOADS = {
    "rqc12": Workload("rqc12", 3, 4, 8, 4, 101, 201, 60, 0,
                      description="12-qubit 3x4 lattice, 8 cycles, 4 open qubits, unsliced"),
    "rqc30": Workload("rqc30", 5, 6, 14, 6, 102, 202, 28, 8,
                      description="30-qubit 5x6 lattice, 14 cycles, 6 open qubits, "
                                  "8 sliced bonds (256 slices), cap 2^28"),
    "rqc30d12": Workload("rqc30d12", 5, 6, 12, 9, 130, 230, 28, 0,
                         description="30-qubit 5x6 lattice, 12 cycles, 9 open qubits, cap 2^28"),
    # the precision form at full size: 53 qubits, largest intermediate 2^30
    "rqc53d12": Workload("rqc53d12", 6, 9, 12, 9, 103, 203, 30, 0, removed=((5, 8),), trials=4,
                         description="53-qubit 6x9 lattice minus one site, 12 cycles, 9 open qubits, "
                                     "sliced to cap 2^30"),
    # the batching form's large network
    "rqc40": Workload("rqc40", 5, 8, 16, 6, 104, 204, 28, 0, trials=4,
                      description="40-qubit 5x8 lattice, 16 cycles, 6 open qubits, sliced to cap 2^28"),
    # the slicing-choice workload of the learned cost model
    "rqc53d14": Workload("rqc53d14", 6, 9, 14, 6, 105, 205, 30, 0, removed=((5, 8),), trials=4,
                         description="53-qubit 6x9 lattice minus one site, 14 cycles, 6 open qubits, "
                                     "sliced to cap 2^30"),
}


@lru_cache(maxsize=None)
def build(name: str):
    """(circuit, network, path dict) of a named workload; deterministic."""
    w = WORKLOADS[name]
    circ = random_circuit(w.rows, w.cols, w.cycles, w.circuit_seed, removed=w.removed)
    open_q, closed = open_and_closed(circ.n_qubits, w.k_open, w.closed_seed)
    net = circuit_network(circ, open_q, closed)
    best = find_path(net, cap_log2=w.cap_log2, n_sliced=w.n_sliced, trials=w.trials,
                     seed=w.circuit_seed)
    return circ, net, best


def uneven_circuits(n: int, seed: int = 1040, open_k: int = 4, cap_log2: int = 22,
                    trials: int = 1):
    """n seeded lattice circuits of uneven size: R x C grids with 16 <= R*C <= 28 and depth
    drawn from 8..14, k open qubits, unsliced.  These stand in for the many independent
    small sub-networks that share the GPU with the slices of a large one.

    Returns a list of (network, path dict); circuit i uses seed + i (circuit),
    seed + 1000 + i (closed bits) and seed + i (path search)."""
    import numpy as np
    shapes = [(r, c) for r in range(2, 8) for c in range(r, 10) if 16 <= r * c <= 28]
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        r, c = shapes[rng.integers(len(shapes))]
        depth = int(rng.integers(8, 15))
        circ = random_circuit(r, c, depth, seed + i)
        oq, cb = open_and_closed(circ.n_qubits, open_k, seed + 1000 + i)
        net = circuit_network(circ, oq, cb)
        best = find_path(net, cap_log2=cap_log2, trials=trials, seed=seed + i)
        out.append((net, best))
    return out


@lru_cache(maxsize=None)
def sparse_state_workload(count: int = 4096, seed: int = 7):
    """The sparse-state workload (Sec. 3.3): the 30-qubit 5x6 lattice circuit of rqc30d12
    (12 cycles, seed 130) with every qubit measured, `count` uniformly random bitstrings
    (seed `seed`; stand-ins for experimental samples), and a randomised greedy path whose
    sizes count merged open bonds by their distinct bitstring restrictions (seed 1302,
    unsliced; largest intermediate 2^32 elements for the default bitstrings).

    Returns (network, path, bitstrings)."""
    from .circuits import sample_bitstrings
    from .paths import greedy_path
    w = WORKLOADS["rqc30d12"]
    circ = random_circuit(w.rows, w.cols, w.cycles, w.circuit_seed)
    oq, _ = open_and_closed(circ.n_qubits, circ.n_qubits, w.closed_seed)
    net = circuit_network(circ, oq, {})
    bits = sample_bitstrings(circ.n_qubits, count, seed)
    path = greedy_path(net.labels, net.open_labels, net.extents(), seed=1302, temperature=0.3, bitstrings=bits)
    return net, path, bits
