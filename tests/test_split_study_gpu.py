"""The dot-product precision study of Sec. 4.2 on the GPU, through the C ABI.

Vectors with random signs and magnitudes log-uniform over 1e-7 .. 1e3 (the paper's
FP16 range), lengths 128 .. 4096.  Each batch of dot products is one contraction
step A[b, k] B[b, k] -> C[b] (b a batch label, k summed) of a two-tensor network:
complex64 runs it on the FP32 kernels, the split precisions on the split MFMA kernels
(split_policy 2) with three products, or one (tn_plan_set_step_terms).

Parity: the split results against oracle/split.py's emulation of the same products
(per-tensor power-of-two scaling, 16-bit round-to-nearest-even split, exact sums);
the GPU may differ only by its FP32 accumulation.  The study itself: the paper finds
3xFP16 as accurate as FP32 (even better), 3xBF16 between FP32 and one 16-bit
product; the test asserts that ordering of the median relative errors.
"""
import numpy as np
import pytest

from oracle import split
from tn_inputs.network import Network
from tn_inputs.vectors import log_uniform_pairs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tn = pytest.importorskip("paper_2310_03978_amd.tn")

COUNT = 256
LENGTHS = (128, 512, 4096)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gpu_dots(A, B, prec, terms=3):
    """Row-wise dots of float32 matrices through a plan: real parts of C[b]."""
    net = Network(tensors=[A.astype(np.complex128), B.astype(np.complex128)], labels=[(0, 1), (0, 1)],
                  open_labels=(0,))
    with tn.Plan(net.tensors, net.labels, net.open_labels, [(0, 1)], precision=prec, split_policy=2) as p:
        st = p.steps()[0]
        if prec != "c64":
            assert st["kernel"] == (2 if prec == "f16x3" else 3), st
            if terms == 1:
                p.set_step_terms(0, 1)
        else:
            assert st["kernel"] in (0, 1), st
        p.contract()
        c, _ = p.amplitudes()
    assert np.all(c.imag == 0)
    return c.real


@pytest.mark.parametrize("length", LENGTHS)
def test_split_dots_match_the_oracle_emulation(length):
    """Every split dot equals the oracle's exact sum of the same rounded, scaled products up
    to FP32 accumulation: the median deviation stays at the FP32 level and no deviation
    exceeds the worst-case FP32 summation bound (k * 2^-24 * sum |terms|)."""
    A, B = log_uniform_pairs(COUNT, length, seed=100 + length)
    scale = np.array([split.abs_dot(a, b) for a, b in zip(A, B)])
    for prec, fmt in (("f16x3", "fp16"), ("bf16x3", "bf16")):
        for terms in (3, 1):
            got = _gpu_dots(A, B, prec, terms)
            want = split.batch_dots(A, B, fmt, terms)
            dev = np.abs(got - want) / scale
            print(f"k={length} {prec} terms={terms}: deviation from the oracle median {np.median(dev):.2e} "
                  f"max {dev.max():.2e}", flush=True)
            assert np.median(dev) <= 2e-6, (prec, terms)
            assert np.all(dev <= length * 2.0 ** -24 * 3), (prec, terms)


def test_precision_study_ordering():
    """Median relative errors against the exact dot products over all lengths: 3xFP16 within
    a factor 2 of FP32, FP32 < 3xBF16 < 1xFP16 < 1xBF16."""
    errs = {}
    for length in LENGTHS:
        A, B = log_uniform_pairs(COUNT, length, seed=200 + length)
        exact = np.array([split.dot_exact(a, b) for a, b in zip(A, B)])
        runs = {"fp32": _gpu_dots(A, B, "c64"), "3xfp16": _gpu_dots(A, B, "f16x3"),
                "3xbf16": _gpu_dots(A, B, "bf16x3"), "1xfp16": _gpu_dots(A, B, "f16x3", 1),
                "1xbf16": _gpu_dots(A, B, "bf16x3", 1)}
        for name, d in runs.items():
            errs.setdefault(name, []).extend((np.abs(d - exact) / np.abs(exact)).tolist())
    med = {k: float(np.median(v)) for k, v in errs.items()}
    print("median relative error: " + ", ".join(f"{k} {v:.2e}" for k, v in med.items()), flush=True)
    assert med["3xfp16"] <= 2 * med["fp32"]
    assert med["fp32"] < med["3xbf16"] < med["1xfp16"] < med["1xbf16"]
