"""Pins of the extended-precision oracle (oracle/split.py, Sec. 4.2) on the CPU.

Each pin checks the oracle against something other than its own code: textbook
rounding cases worked by hand, torch's float32 -> bfloat16 / float16 conversions (a
second library), the error bound of a two-term split, exact integer arithmetic, and
the algebra of the dropped lo * lo term.
"""
import math

import numpy as np
import pytest

from oracle import split
from tn_inputs.vectors import log_uniform_pairs


def test_ties_round_to_even_by_hand():
    # fp16 keeps 10 fraction bits: 1 + 2^-11 lies halfway between 1 and 1 + 2^-10 -> 1 (even);
    # 1 + 3 * 2^-11 lies halfway between 1 + 2^-10 and 1 + 2^-9 -> 1 + 2^-9 (even)
    assert split.round16(np.float32(1 + 2.0 ** -11), "fp16") == 1.0
    assert split.round16(np.float32(1 + 3 * 2.0 ** -11), "fp16") == 1 + 2.0 ** -9
    assert split.round16(np.float32(1 + 2.0 ** -11 + 2.0 ** -20), "fp16") == 1 + 2.0 ** -10
    # bf16 keeps 7 fraction bits: the same pattern two decades up
    assert split.round16(np.float32(1 + 2.0 ** -8), "bf16") == 1.0
    assert split.round16(np.float32(1 + 3 * 2.0 ** -8), "bf16") == 1 + 2.0 ** -6
    assert split.round16(np.float32(-(1 + 2.0 ** -8 + 2.0 ** -20)), "bf16") == -(1 + 2.0 ** -7)


def test_rounding_matches_torch_conversions():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    xb = x[np.abs(x) < 3e38]
    ref_b = torch.from_numpy(xb).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(split.round16(xb, "bf16"), ref_b)
    xh = x[np.abs(x) < 65504]   # fp16 range (subnormals included)
    ref_h = torch.from_numpy(xh).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_array_equal(split.round16(xh, "fp16"), ref_h)


@pytest.mark.parametrize("fmt,p", [("fp16", 11), ("bf16", 8)])
def test_split_error_bound(fmt, p):
    """Two roundings to a p-bit significand: |x - hi| <= 2^-p |x| and |x - hi - lo| <=
    2^-p |x - hi| <= 2^-2p |x| (normal range of the 16-bit format)."""
    rng = np.random.default_rng(p)
    x = (rng.uniform(1.0, 2.0, 100000) * 2.0 ** rng.integers(3, 15, 100000)).astype(np.float32)
    x *= np.where(rng.integers(0, 2, x.size) == 1, 1, -1).astype(np.float32)
    hi, lo = split.split(x, fmt)
    xd = x.astype(np.float64)
    assert np.all(np.abs(xd - hi) <= 2.0 ** -p * np.abs(xd))
    assert np.all(np.abs(xd - hi - lo) <= 2.0 ** (-2 * p) * np.abs(xd))


def test_split_is_exact_for_short_significands():
    """x with at most 22 significant bits (two fp16 significands) splits exactly."""
    x = np.array([1 + 2.0 ** -12 + 2.0 ** -21, -(3 + 2.0 ** -15), 2.0 ** 10 * (1 + 2.0 ** -13)],
                 dtype=np.float32)
    hi, lo = split.split(x, "fp16")
    np.testing.assert_array_equal(hi + lo, x.astype(np.float64))
    np.testing.assert_array_equal(hi, [1.0, -3.0, 2.0 ** 10])


def test_scale_exponent_puts_the_maximum_in_range():
    for m in (1.0, 3e-7, 1e3, 2.0 ** 14, 2.0 ** 15 - 1, 0.7):
        s = split.scale_exponent(np.array([m, -m / 3], dtype=np.float32))
        assert 2.0 ** 14 <= float(np.float32(m)) * 2.0 ** s < 2.0 ** 15
    assert split.scale_exponent(np.zeros(4)) == 0


def test_integer_dots_are_exact():
    """Small integers are exact in both 16-bit formats: lo = 0 and every split dot equals
    the exact dot (the power-of-two scaling is exact too)."""
    rng = np.random.default_rng(8)
    a = rng.integers(-100, 101, 512).astype(np.float32)
    b = rng.integers(-100, 101, 512).astype(np.float32)
    exact = float(np.dot(a.astype(np.int64), b.astype(np.int64)))
    for fmt in split.FORMATS:
        for terms in (1, 3, 4):
            assert split.dot(a, b, fmt, terms) == exact


def test_dropped_term_is_lo_times_lo():
    a, b = log_uniform_pairs(1, 1024, seed=4)
    a, b = a[0], b[0]
    for fmt in split.FORMATS:
        sa, sb = split.scale_exponent(a), split.scale_exponent(b)
        _, la = split.split(np.ldexp(a.astype(np.float64), sa).astype(np.float32), fmt)
        _, lb = split.split(np.ldexp(b.astype(np.float64), sb).astype(np.float32), fmt)
        d4, d3 = split.dot(a, b, fmt, 4), split.dot(a, b, fmt, 3)
        want = math.ldexp(math.fsum((la * lb).tolist()), -(sa + sb))
        # each dot is correctly rounded to FP64: their difference is exact up to two roundings
        assert abs((d4 - d3) - want) <= 2 * 2.0 ** -52 * max(abs(d4), abs(d3))
        assert want != 0.0


def test_study_ordering_of_the_emulated_methods():
    """The Sec. 4.2 study on the oracle alone: on the FP16 range, three bf16 products are
    less accurate than three fp16 products and more accurate than one product of either."""
    A, B = log_uniform_pairs(64, 1024, seed=11)
    exact = np.array([split.dot_exact(a, b) for a, b in zip(A, B)])

    def err(fmt, terms):
        d = split.batch_dots(A, B, fmt, terms)
        return float(np.median(np.abs(d - exact) / np.abs(exact)))

    e = {(f, t): err(f, t) for f in split.FORMATS for t in (1, 3)}
    assert e[("fp16", 3)] < e[("bf16", 3)] < e[("bf16", 1)]
    assert e[("bf16", 3)] < e[("fp16", 1)] < e[("bf16", 1)]
