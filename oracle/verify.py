"""Verification measures of random-circuit sampling in FP64: LXEB, its error, Porter-Thomas.

TEST INFRASTRUCTURE ONLY (checks the library's XEB statistics kernel).

* lxeb(p, n)          F_l = 2^N (1/m) sum_i p_U(x_i) - 1 over m sampled bitstrings x_i with
                      ideal probabilities p_U(x_i) (Sec. 2.2, the sampled LXEB equation)
* lxeb_amplitudes     the same through the squared L2 norm of the m amplitudes:
                      F_l = L2(x)^2 2^N / m - 1 (Sec. 4.3)
* eps_fl(eps, F)      relative error of F_l implied by a relative error eps of the squared
                      norm: eps_Fl = eps_L2^2 (1 + F_l) / F_l (Sec. 4.3)
* pt_density(x, F)    the density of x = log(D p) for bitstrings sampled with fidelity F
                      from a Porter-Thomas distribution: (1 + F (e^x - 1)) e^(x - e^x),
                      D = 2^N (Sec. 5.1)
* pt_cdf, pt_bin_probs  that density integrated (closed form) and over histogram bins
"""
from __future__ import annotations

import math

import numpy as np


def lxeb(probs, n_qubits: int) -> float:
    p = np.asarray(probs, dtype=np.float64)
    return float(2.0 ** n_qubits * math.fsum(p.tolist()) / p.size - 1.0)


def lxeb_amplitudes(amps, n_qubits: int) -> float:
    a = np.asarray(amps, dtype=np.complex128)
    l2sq = math.fsum((a.real ** 2).tolist()) + math.fsum((a.imag ** 2).tolist())
    return float(l2sq * 2.0 ** n_qubits / a.size - 1.0)


def eps_fl(eps_l2sq: float, f_l: float) -> float:
    return float(eps_l2sq * (1.0 + f_l) / f_l)


def pt_density(x, fidelity: float):
    x = np.asarray(x, dtype=np.float64)
    return (1.0 + fidelity * np.expm1(x)) * np.exp(x - np.exp(x))


def pt_cdf(x, fidelity: float):
    """Closed form of the integral of pt_density from -inf to x: with u = e^x,
    int e^(x - e^x) dx = 1 - e^-u and int e^(2x - e^x) dx = 1 - (1 + u) e^-u, so
    C(x) = (1 - F)(1 - e^-u) + F (1 - (1 + u) e^-u)."""
    u = np.exp(np.asarray(x, dtype=np.float64))
    a = -np.expm1(-u)
    # 1 - (1 + u) e^-u cancels for small u: there its Taylor series u^2/2 - u^3/3 + u^4/8 - ...
    with np.errstate(over="ignore"):
        direct = -np.expm1(-u) - u * np.exp(-u)
    series = u * u * (0.5 - u * (1.0 / 3.0 - u * (0.125 - u / 30.0)))
    b = np.where(u < 1e-2, series, direct)
    return (1.0 - fidelity) * a + fidelity * b


def pt_bin_probs(edges, fidelity: float):
    c = pt_cdf(np.asarray(edges, dtype=np.float64), fidelity)
    return np.diff(c)
