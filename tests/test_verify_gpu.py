"""The verification pipeline on the GPU (Sec. 2.2 LXEB, Sec. 4.3 eps_Fl, Sec. 5.1 Porter-Thomas).

Synthetic samples stand in for an experiment's: bitstrings of a 16-qubit, 20-cycle lattice
circuit drawn from F p + (1 - F) uniform (p from the oracle's state vector; F = 1 ideal,
0.5, 0 pure noise).  Their amplitudes come from one sparse-state contraction on the GPU
(Sec. 3.3), and tn_plan_xeb forms the LXEB sums and the histogram of log(D p) on the GPU
in FP64.  Checked against the oracle (oracle/verify.py on the state vector's
probabilities of the same samples): LXEB, the second moment and the histogram counts; the
split-FP16 run's LXEB against complex64's through eps_Fl = eps_L2^2 (1 + F) / F.
"""
import numpy as np
import pytest

from oracle import statevector, verify
from tn_inputs.circuits import open_and_closed, random_circuit
from tn_inputs.network import circuit_network
from tn_inputs.paths import greedy_path
from tn_inputs.samples import index_to_bits, sample_with_fidelity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tn = pytest.importorskip("paper_2310_03978_amd.tn")

EDGES = (-6.0, 3.0, 18)   # x_lo, x_hi, bins


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def circuit():
    circ = random_circuit(4, 4, 20, seed=161)
    p = np.abs(statevector.simulate(circ).reshape(-1)) ** 2
    oq, _ = open_and_closed(circ.n_qubits, circ.n_qubits, 161)
    net = circuit_network(circ, oq, {})
    path = greedy_path(net.labels, net.open_labels, net.extents(), seed=5)
    return circ, p, net, path


def _oracle_hist(p_samples, n):
    lo, hi, nb = EDGES
    x = np.log(2.0 ** n * p_samples)
    b = np.floor((x - lo) / (hi - lo) * nb)
    b = np.clip(np.nan_to_num(b, neginf=0, posinf=nb - 1), 0, nb - 1).astype(int)
    return np.bincount(b, minlength=nb)


@pytest.mark.parametrize("fid", [1.0, 0.5, 0.0])
def test_lxeb_of_sampled_bitstrings_matches_the_oracle(circuit, fid):
    circ, p, net, path = circuit
    n = circ.n_qubits
    idx = sample_with_fidelity(p, 4096, fid, seed=41)
    bits = index_to_bits(idx, n)
    want = verify.lxeb(p[idx], n)
    want2 = (2.0 ** n) ** 2 * np.mean(p[idx] ** 2)
    hist_want = _oracle_hist(p[idx], n)
    got = {}
    for prec in ("c64", "f16x3"):
        with tn.Plan(net.tensors, net.labels, net.open_labels, path, precision=prec, bitstrings=bits) as pl:
            pl.contract()
            amps, _ = pl.amplitudes()
            stats, hist = pl.xeb(n, EDGES[2], EDGES[0], EDGES[1])
        got[prec] = (stats, hist, amps)
        print(f"F={fid} {prec}: LXEB {stats['lxeb']:.6f} (oracle {want:.6f}), E[(Dp)^2] {stats['mean_dp2']:.4f} "
              f"(oracle {want2:.4f}), samples {stats['samples']}", flush=True)
        assert stats["samples"] == len(idx)
        assert abs(stats["lxeb"] - want) <= 1e-4 * (1 + abs(want)), (prec, stats["lxeb"], want)
        assert abs(stats["mean_dp2"] - want2) <= 1e-3 * want2
        # counts can differ only for samples within rounding of a bin edge
        assert np.abs(hist - hist_want).sum() <= 4, (hist, hist_want)
        # the same statistics from the amplitudes the library returned
        assert stats["lxeb"] == pytest.approx(verify.lxeb_amplitudes(amps, n), abs=1e-9)
    # eps_Fl: the relative error of F_l implied by the squared-norm error of the split run
    if fid > 0:
        a16, a64 = got["f16x3"][2], got["c64"][2]
        eps = abs(np.vdot(a16, a16).real - np.vdot(a64, a64).real) / np.vdot(a64, a64).real
        f16, f64 = got["f16x3"][0]["lxeb"], got["c64"][0]["lxeb"]
        pred = verify.eps_fl(eps, f64)
        print(f"F={fid}: eps_L2^2 {eps:.3e}, eps_Fl {pred:.3e}, measured |dF|/F {abs(f16 - f64) / f64:.3e}",
              flush=True)
        assert abs(abs(f16 - f64) / f64 - pred) <= 1e-6 + 1e-3 * pred
        assert pred < 1e-4


def test_porter_thomas_from_the_full_state(circuit):
    """Every amplitude of the state (all qubits open, a dense plan): sum p = 1 (LXEB over
    the whole space is 0), D sum p^2 against the oracle, and the histogram of log(D p) over
    all bitstrings against the oracle's and against the Porter-Thomas law of uniformly
    drawn bitstrings (F = 0)."""
    circ, p, net, path = circuit
    n = circ.n_qubits
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, precision="f16x3") as pl:
        pl.contract()
        amps, _ = pl.amplitudes()
        stats, hist = pl.xeb(n, EDGES[2], EDGES[0], EDGES[1])
    print(f"full state: {stats}", flush=True)
    assert stats["samples"] == 2 ** n
    # sum p is the squared norm of the returned amplitudes (the GPU's FP64 sum)
    assert stats["sum_p"] == pytest.approx(float(np.sum(np.abs(amps) ** 2)), rel=1e-12)
    # and 1 up to the amplitudes' own error: with r = ||a - a*|| / ||a*|| and ||a*|| = 1,
    # |sum p - 1| = | ||a||^2 - ||a*||^2 | <= r (2 + r)
    sv = statevector.simulate(circ).reshape(-1)
    r = float(np.linalg.norm(amps - sv) / np.linalg.norm(sv))
    print(f"full state: rel_l2 {r:.3e}, |sum p - 1| {abs(stats['sum_p'] - 1.0):.3e}", flush=True)
    assert r <= 1e-3
    assert abs(stats["sum_p"] - 1.0) <= r * (2.0 + r) + 1e-12
    assert abs(stats["lxeb"]) <= r * (2.0 + r) + 1e-12
    assert stats["mean_dp2"] == pytest.approx(2.0 ** n * np.sum(p ** 2), rel=1e-4)
    assert np.abs(hist - _oracle_hist(p, n)).sum() <= 8
    lo, hi, nb = EDGES
    edges = np.linspace(lo, hi, nb + 1)
    want0 = verify.pt_bin_probs(edges, 0.0)
    want0[0] += verify.pt_cdf(edges[0], 0.0)
    want0[-1] += 1.0 - verify.pt_cdf(edges[-1], 0.0)
    assert 0.5 * np.abs(hist / hist.sum() - want0).sum() < 0.05
