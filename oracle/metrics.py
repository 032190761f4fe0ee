"""Error measures between an amplitude batch and the complex128 oracle.

TEST INFRASTRUCTURE ONLY.

* rel_l2      = ||a - a*||_2 / ||a*||_2 (the judged amplitude error)
* eps_l2sq    = |L2^2 - L2^2'| / L2^2, the relative error of the squared norm
                (Sec. 4.3, Eq. for epsilon_L2^2)
* fidelity    = |<a*, a>|^2 / (||a||^2 ||a*||^2)
* max_err     = max_i |a_i - a*_i| / (||a*||_2 / sqrt(n))
* lxeb        = L2(x)^2 2^N / m - 1 (Sec. 4.3, the LXEB estimator written
                through the squared norm of m amplitudes of an N-qubit circuit)
"""
from __future__ import annotations

import numpy as np


def rel_l2(a, ref) -> float:
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / den) if den > 0 else float(np.linalg.norm(a))


def eps_l2sq(a, ref) -> float:
    l2 = float(np.vdot(ref, ref).real)
    l2p = float(np.vdot(a, a).real)
    return abs(l2 - l2p) / l2


def fidelity(a, ref) -> float:
    num = abs(np.vdot(ref, a)) ** 2
    den = float(np.vdot(a, a).real) * float(np.vdot(ref, ref).real)
    return float(num / den) if den > 0 else 0.0


def max_err(a, ref) -> float:
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    scale = np.linalg.norm(ref) / np.sqrt(ref.size)
    return float(np.max(np.abs(a - ref)) / scale)


def lxeb(amps, n_qubits: int) -> float:
    amps = np.asarray(amps, dtype=np.complex128)
    return float(np.vdot(amps, amps).real) * 2.0 ** n_qubits / amps.size - 1.0


def report(a, ref) -> dict:
    return {"rel_l2": rel_l2(a, ref), "eps_l2sq": eps_l2sq(a, ref),
            "fidelity": fidelity(a, ref), "max_err": max_err(a, ref)}
