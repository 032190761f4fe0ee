"""Write the oracle's amplitudes of the 30-qubit, 12-cycle workload to a text fixture.

    python tests/golden/make_rqc30d12_amplitudes.py

Calls only the CPU oracle (complex128 pairwise contraction along the workload's path)
on the seeded network from tn_inputs; takes about a minute on 8 cores.  The fixture
records a SHA-256 of the network and path so that a test can tell when the input
generator has changed and the fixture must be rewritten.
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import contract  # noqa: E402
from tn_inputs import configs  # noqa: E402

NAME = "rqc30d12"
PATH = os.path.join(HERE, "rqc30d12_amplitudes.txt")


def network_digest(net, best) -> str:
    h = hashlib.sha256()
    for t, lab in zip(net.tensors, net.labels):
        h.update(np.ascontiguousarray(t, dtype=np.complex128).tobytes())
        h.update(repr(tuple(int(x) for x in lab)).encode())
    h.update(repr(tuple(int(x) for x in net.open_labels)).encode())
    h.update(repr(tuple((int(i), int(j)) for i, j in best["path"])).encode())
    return h.hexdigest()


def read_fixture(path: str = PATH):
    """(digest, amplitudes) of the fixture."""
    digest, vals = None, []
    with open(path) as f:
        for line in f:
            if line.startswith("# network sha256:"):
                digest = line.split(":", 1)[1].strip()
            elif line.strip() and not line.startswith("#"):
                re, im = line.split()
                vals.append(complex(float(re), float(im)))
    return digest, np.array(vals, dtype=np.complex128)


def main():
    _, net, best = configs.build(NAME)
    amps = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    with open(PATH, "w") as f:
        f.write(f"# {configs.WORKLOADS[NAME].description}\n")
        f.write("# oracle amplitudes (complex128), open qubits in network order, one 're im' per line\n")
        f.write(f"# network sha256: {network_digest(net, best)}\n")
        for a in amps:
            f.write(f"{a.real:.17e} {a.imag:.17e}\n")
    print(f"wrote {PATH}: {amps.size} amplitudes")


if __name__ == "__main__":
    main()
