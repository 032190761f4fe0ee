"""Extended-precision products of Sec. 4.2 in FP64: the hi/lo split and split dot products.

TEST INFRASTRUCTURE ONLY (checks the library's split-precision kernels).

The paper's 3-product method (the 3xTF32 equation of Sec. 4.2, carried over to
FP16 and BF16 in the same section): an FP32 operand x becomes
    hi = round(x),  lo = round(x - hi)
in the 16-bit format, and a product a * b is approximated by
    hi_a hi_b + hi_a lo_b + lo_a hi_b
(lo_a lo_b is dropped).  Rounding is to nearest, ties to even (the reading of the
equation's unbalanced parenthesis taken here: lo rounds the exact residual).

Dynamic scaling (Sec. 4.2, last paragraph; the re-scaling outlook of Sec. 6): FP16
covers a narrow exponent range, so a whole operand (vector or tensor) is first
multiplied by one power of two 2^s that puts its largest magnitude in
[2^14, 2^15); the result is multiplied by 2^-(s_a + s_b).  BF16 takes the same
scaling (harmless: powers of two are exact).

Every function here computes in FP64 or exactly (``math.fsum``), so its only
rounding is the 16-bit rounding the method itself prescribes: products of two
16-bit values are exact in FP64 and the sums below are exactly rounded.
"""
from __future__ import annotations

import math

import numpy as np

FORMATS = ("fp16", "bf16")
TARGET_EXP = 14   # largest magnitude after scaling lies in [2^14, 2^15)


def round16(x, fmt: str) -> np.ndarray:
    """Round float32 values to the 16-bit format (nearest, ties to even), as float64."""
    x = np.asarray(x, dtype=np.float32)
    if fmt == "fp16":
        return x.astype(np.float16).astype(np.float64)
    if fmt != "bf16":
        raise ValueError(fmt)
    # bf16 keeps the top 16 bits of the float32 pattern; round the dropped 16 bits to
    # nearest with ties to even by adding 0x7fff plus the lowest kept bit
    bits = x.view(np.uint32).astype(np.uint64)
    keep_lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + keep_lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def scale_exponent(x) -> int:
    """s such that max|x| * 2^s lies in [2^TARGET_EXP, 2^(TARGET_EXP + 1)); 0 for all-zero x."""
    m = float(np.max(np.abs(np.asarray(x, dtype=np.float64)))) if np.size(x) else 0.0
    if m == 0.0 or not math.isfinite(m):
        return 0
    _, e = math.frexp(m)          # m = f 2^e, f in [0.5, 1): m in [2^(e-1), 2^e)
    return TARGET_EXP - (e - 1)


def split(x, fmt: str):
    """(hi, lo) of float32 values x (no scaling): hi = round(x), lo = round(x - hi).

    x - hi is formed in FP64, where it is exact."""
    x = np.asarray(x, dtype=np.float32)
    hi = round16(x, fmt)
    lo = round16((x.astype(np.float64) - hi).astype(np.float32), fmt)
    return hi, lo


def scaled_split(x, fmt: str):
    """(hi, lo, s): the split of x * 2^s with s = scale_exponent(x)."""
    x = np.asarray(x, dtype=np.float32)
    s = scale_exponent(x)
    xs = np.ldexp(x.astype(np.float64), s).astype(np.float32)   # exact (a power of two)
    hi, lo = split(xs, fmt)
    return hi, lo, s


def dot(a, b, fmt: str, terms: int = 3, sa: int | None = None, sb: int | None = None) -> float:
    """Split dot product of float32 vectors a, b.

    a is scaled by 2^sa and b by 2^sb before the split; by default each vector's own
    scale_exponent (pass the exponent of a whole tensor for per-tensor scaling).
    terms = 3: sum of hi_a hi_b + hi_a lo_b + lo_a hi_b; terms = 1: sum of hi_a hi_b;
    terms = 4: all four products (lo_a lo_b kept).  Summed exactly, then scaled back."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    sa = scale_exponent(a) if sa is None else sa
    sb = scale_exponent(b) if sb is None else sb
    ha, la = split(np.ldexp(a.astype(np.float64), sa).astype(np.float32), fmt)
    hb, lb = split(np.ldexp(b.astype(np.float64), sb).astype(np.float32), fmt)
    parts = [ha * hb]
    if terms >= 3:
        parts += [ha * lb, la * hb]
    if terms == 4:
        parts.append(la * lb)
    if terms not in (1, 3, 4):
        raise ValueError(terms)
    return math.ldexp(math.fsum(np.concatenate(parts).tolist()), -(sa + sb))


def batch_dots(A, B, fmt: str, terms: int = 3) -> np.ndarray:
    """Row-wise split dot products of float32 matrices A, B (count x length) with one scale
    per matrix (per-tensor scaling, as for a tensor operand of a contraction step)."""
    sa, sb = scale_exponent(A), scale_exponent(B)
    return np.array([dot(a, b, fmt, terms, sa, sb) for a, b in zip(A, B)])


def dot_exact(a, b) -> float:
    """The dot product of the float32 inputs, correctly rounded to FP64."""
    a = np.asarray(a, dtype=np.float32).astype(np.float64)
    b = np.asarray(b, dtype=np.float32).astype(np.float64)
    return math.fsum((a * b).tolist())   # float32 x float32 is exact in FP64


def abs_dot(a, b) -> float:
    """sum |a_i b_i|: the scale of the rounding error bounds of any summation order."""
    a = np.asarray(a, dtype=np.float32).astype(np.float64)
    b = np.asarray(b, dtype=np.float32).astype(np.float64)
    return math.fsum(np.abs(a * b).tolist())
