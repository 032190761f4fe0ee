"""Seeded random quantum circuits on 2D lattices (input generator only).

The circuit family follows the random-circuit-sampling description of the
paper (Sec. 2.2): each cycle is a layer of single-qubit gates chosen at random
from {sqrt(X), sqrt(Y), sqrt(W)} followed by a layer of fSim two-qubit gates.
The paper names the gates but gives neither matrices, the coupler pattern nor
the fSim angles; the readings used here are:

* sqrt(X) = (1/sqrt2) [[1, -i], [-i, 1]]
* sqrt(Y) = (1/sqrt2) [[1, -1], [1, 1]]
* sqrt(W) = (1/sqrt2) [[1, -e^{i pi/4}], [e^{-i pi/4}, 1]]
* fSim(theta, phi) = [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,e^{-i phi}]]
  with theta ~ U(0, pi/2), phi ~ U(0, pi/3) drawn per gate.
* Qubits are lattice sites numbered row-major.  Couplers come in four
  classes: A = (r,c)-(r,c+1) with c even, B = the same with c odd,
  C = (r,c)-(r+1,c) with r even, D = the same with r odd.  Cycle t uses class
  (t + off) mod 4 in the order A, B, C, D; ``off`` is drawn from the seed.
* Single-qubit gates are drawn i.i.d. uniformly per qubit and cycle
  (``no_repeat=True`` forbids repeating the previous gate on a qubit).
* There is no extra single-qubit layer after the last cycle.

Two-qubit gate matrices act on the basis index 2*x_a + x_b where (a, b) is the
gate's qubit pair in the stored order.  This module holds no contraction
arithmetic: it only produces gate lists.  Random numbers come from numpy's
PCG64 generator (``numpy.random.default_rng``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_S2 = 1.0 / np.sqrt(2.0)

SQRT_X = _S2 * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)
SQRT_Y = _S2 * np.array([[1, -1], [1, 1]], dtype=np.complex128)
SQRT_W = _S2 * np.array([[1, -np.exp(1j * np.pi / 4)],
                         [np.exp(-1j * np.pi / 4), 1]], dtype=np.complex128)
SINGLE_QUBIT_GATES = {"sqrt_x": SQRT_X, "sqrt_y": SQRT_Y, "sqrt_w": SQRT_W}
_SQ_NAMES = ("sqrt_x", "sqrt_y", "sqrt_w")


def fsim(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi) in the basis |00>, |01>, |10>, |11>."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


@dataclass
class Gate:
    name: str
    qubits: tuple          # (q,) or (qa, qb)
    matrix: np.ndarray     # 2x2 or 4x4 complex128
    cycle: int


@dataclass
class Circuit:
    n_qubits: int
    sites: list            # (row, col) of each qubit, row-major order
    gates: list = field(default_factory=list)
    cycles: int = 0
    seed: int = 0


def lattice_sites(rows: int, cols: int, removed=()) -> list:
    removed = set(tuple(x) for x in removed)
    return [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in removed]


def coupler_classes(sites: list) -> list:
    """The four coupler classes A, B, C, D as lists of qubit-index pairs."""
    index = {s: i for i, s in enumerate(sites)}
    classes = [[], [], [], []]
    for (r, c), q in index.items():
        right = index.get((r, c + 1))
        if right is not None:
            classes[0 if c % 2 == 0 else 1].append((q, right))
        down = index.get((r + 1, c))
        if down is not None:
            classes[2 if r % 2 == 0 else 3].append((q, down))
    for cl in classes:
        cl.sort()
    return classes


def random_circuit(rows: int, cols: int, cycles: int, seed: int, removed=(),
                   no_repeat: bool = False) -> Circuit:
    """Random circuit on a rows x cols lattice (minus ``removed`` sites)."""
    rng = np.random.default_rng(seed)
    sites = lattice_sites(rows, cols, removed)
    n = len(sites)
    classes = coupler_classes(sites)
    offset = int(rng.integers(0, 4))
    circ = Circuit(n_qubits=n, sites=sites, cycles=cycles, seed=seed)
    last = [-1] * n
    for t in range(cycles):
        for q in range(n):
            if no_repeat and last[q] >= 0:
                choice = int(rng.integers(0, 2))
                g = [i for i in range(3) if i != last[q]][choice]
            else:
                g = int(rng.integers(0, 3))
            last[q] = g
            name = _SQ_NAMES[g]
            circ.gates.append(Gate(name, (q,), SINGLE_QUBIT_GATES[name], t))
        for (qa, qb) in classes[(t + offset) % 4]:
            theta = rng.uniform(0.0, np.pi / 2)
            phi = rng.uniform(0.0, np.pi / 3)
            circ.gates.append(Gate("fsim", (qa, qb), fsim(theta, phi), t))
    return circ


def product_circuit(n_qubits: int, names) -> Circuit:
    """One single-qubit gate per qubit (closed-form test circuits)."""
    circ = Circuit(n_qubits=n_qubits, sites=[(0, q) for q in range(n_qubits)], cycles=1)
    for q, name in enumerate(names):
        circ.gates.append(Gate(name, (q,), SINGLE_QUBIT_GATES[name], 0))
    return circ


def open_and_closed(n_qubits: int, k_open: int, seed: int):
    """Open qubits are the last k (row-major); the rest get seeded random bits."""
    rng = np.random.default_rng(seed)
    open_q = tuple(range(n_qubits - k_open, n_qubits))
    closed = {q: int(b) for q, b in zip(range(n_qubits - k_open),
                                         rng.integers(0, 2, size=n_qubits - k_open))}
    return open_q, closed


def sample_bitstrings(n_qubits: int, count: int, seed: int, duplicates: int = 0):
    """count uniformly random bitstrings (uint8 [count, n_qubits], qubit order), seeded;
    the last `duplicates` rows repeat earlier ones.  Stand-ins for measured samples."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2, size=(count, n_qubits), dtype=np.uint8)
    if duplicates:
        src = rng.integers(0, max(count - duplicates, 1), size=duplicates)
        x[count - duplicates:] = x[src]
    return x
