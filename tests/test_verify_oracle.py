"""Pins of the verification oracle (oracle/verify.py): LXEB, eps_Fl, the Porter-Thomas law.

Each pin checks against something other than the formula it tests: a worked example by
hand, the behaviour of the estimator on samples whose expectation is known exactly from
the state vector, the Porter-Thomas density against its own closed-form integral and
moments derived by hand, and the error propagation against a direct perturbation.
"""
import numpy as np
import pytest

from oracle import statevector, verify
from tn_inputs.circuits import random_circuit
from tn_inputs.samples import index_to_bits, sample_with_fidelity


def test_lxeb_worked_example():
    """N = 1, ideal probabilities p(0) = 3/4, p(1) = 1/4, samples 0, 0, 1:
    F = 2 (3/4 + 3/4 + 1/4) / 3 - 1 = 1/6, also through the amplitudes' squared norm."""
    p = {0: 0.75, 1: 0.25}
    samples = [0, 0, 1]
    assert verify.lxeb([p[x] for x in samples], 1) == pytest.approx(1 / 6, abs=1e-15)
    amps = [np.sqrt(p[x]) * np.exp(1j * x) for x in samples]
    assert verify.lxeb_amplitudes(amps, 1) == pytest.approx(1 / 6, abs=1e-15)


def test_eps_fl_matches_a_direct_perturbation():
    """Scaling every amplitude by sqrt(1 + eps) changes L2^2 by the relative error eps; the
    LXEB estimate then moves by exactly eps_Fl * F."""
    rng = np.random.default_rng(2)
    a = (rng.standard_normal(4096) + 1j * rng.standard_normal(4096)) * 2.0 ** -10
    f = verify.lxeb_amplitudes(a, 20)
    for eps in (1e-3, 3.36e-5):
        f2 = verify.lxeb_amplitudes(a * np.sqrt(1 + eps), 20)
        assert abs(f2 - f) / f == pytest.approx(verify.eps_fl(eps, f), rel=1e-6)


@pytest.mark.parametrize("fid", [0.0, 0.00248, 0.5, 1.0])
def test_porter_thomas_density_integrals(fid):
    """The density integrates to 1; its closed-form integral is its antiderivative; and
    E[e^x] = E[D p] = 1 + F (ideal samples of a Porter-Thomas state give D sum p^2 = 2,
    uniform ones 1; a fidelity-F mixture the weighted mean)."""
    x = np.linspace(-30.0, 4.0, 400001)
    dens = verify.pt_density(x, fid)
    dx = x[1] - x[0]
    assert np.trapezoid(dens, x) == pytest.approx(1.0, abs=1e-6)
    assert np.trapezoid(np.exp(x) * dens, x) == pytest.approx(1.0 + fid, abs=1e-6)
    c = verify.pt_cdf(x, fid)
    assert c[-1] == pytest.approx(1.0, abs=1e-6) and c[0] == pytest.approx(0.0, abs=1e-12)
    np.testing.assert_allclose(np.gradient(c, dx)[1:-1], dens[1:-1], atol=1e-6)
    assert np.all(verify.pt_bin_probs(x[::1000], fid) >= 0)


@pytest.fixture(scope="module")
def deep16():
    circ = random_circuit(4, 4, 20, seed=161)
    psi = statevector.simulate(circ).reshape(-1)
    return circ, np.abs(psi) ** 2


@pytest.mark.parametrize("fid", [1.0, 0.5, 0.0])
def test_lxeb_estimates_the_fidelity_of_mixture_samples(deep16, fid):
    """Samples of a 16-qubit, 20-cycle circuit drawn from F p + (1 - F) uniform: the LXEB
    estimator's expectation is F (D sum p^2 - 1) exactly; the estimate lies within 5
    standard errors of it (and D sum p^2 is close to Porter-Thomas' 2)."""
    circ, p = deep16
    n = circ.n_qubits
    D = 2.0 ** n
    m = 20000
    idx = sample_with_fidelity(p, m, fid, seed=31)
    est = verify.lxeb(p[idx], n)
    mean_ideal = D * np.sum(p ** 2) - 1.0
    assert abs(mean_ideal - 1.0) < 0.1
    # variance of D p(x) under the mixture
    e1 = fid * D * np.sum(p ** 2) + (1 - fid) * 1.0
    e2 = fid * D ** 2 * np.sum(p ** 3) + (1 - fid) * D * np.sum(p ** 2)
    se = np.sqrt((e2 - e1 ** 2) / m)
    assert abs(est - fid * mean_ideal) <= 5 * se, (est, fid * mean_ideal, se)


def test_histogram_of_ideal_samples_follows_porter_thomas(deep16):
    """log(D p) of ideal samples against the F = 1 density integrated over 24 bins: total
    variation distance below 0.03 (and above it for the uniform-sample density)."""
    circ, p = deep16
    n = circ.n_qubits
    idx = sample_with_fidelity(p, 50000, 1.0, seed=7)
    x = np.log(2.0 ** n * p[idx])
    edges = np.linspace(-6.0, 3.0, 25)
    counts, _ = np.histogram(np.clip(x, edges[0], edges[-1] - 1e-12), bins=edges)
    emp = counts / counts.sum()
    want1 = verify.pt_bin_probs(edges, 1.0)
    want1[0] += verify.pt_cdf(edges[0], 1.0)
    want1[-1] += 1.0 - verify.pt_cdf(edges[-1], 1.0)
    want0 = verify.pt_bin_probs(edges, 0.0)
    want0[0] += verify.pt_cdf(edges[0], 0.0)
    want0[-1] += 1.0 - verify.pt_cdf(edges[-1], 0.0)
    assert 0.5 * np.abs(emp - want1).sum() < 0.03
    assert 0.5 * np.abs(emp - want0).sum() > 0.1


def test_bits_of_state_indices():
    np.testing.assert_array_equal(index_to_bits([0, 5, 15], 4),
                                  [[0, 0, 0, 0], [0, 1, 0, 1], [1, 1, 1, 1]])
