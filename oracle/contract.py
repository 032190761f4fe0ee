"""CPU complex128 oracle for sliced pairwise tensor-network contraction.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark; never by the GPU product path.

What it computes (the plain definition, Sec. 2.4 and Sec. 3.1-3.2 of the paper):
for leaves T_1..T_n with label tuples and open labels O,

    a[o] = sum over every non-open label of  prod_t T_t[labels_t].

The path form follows Sec. 3.1: the network is contracted pairwise along a
list of (i, j) slot pairs; each step computes the einsum of Eq. (2.4),
C_gamma = sum_delta A_alpha B_beta, and stores C in slot i while slot j dies.
A label of the pair survives into C when it is open or still appears on
another live tensor; a label shared by A and B that survives is a batch label
(carried, not summed); every other label of A or B is summed.  A label that
appears on only one operand and nowhere else is summed over that operand
before the product.

Slicing (Sec. 3.2): fixing every sliced label to a value splits the
contraction into independent sub-tasks whose results add up to a.  Slice ids
are mixed-radix numbers over the sliced labels, the first sliced label being
the most significant digit; ``amplitudes`` sums slices in increasing id order.

numpy's tensordot (a BLAS complex GEMM) serves as the pairwise product.
"""
from __future__ import annotations

import itertools

import numpy as np


def slice_values(sliced_labels, extents: dict, slice_id: int) -> dict:
    """Mixed-radix decode of a slice id (first sliced label most significant)."""
    vals = {}
    rem = int(slice_id)
    for l in reversed(list(sliced_labels)):
        e = extents[l]
        vals[l] = rem % e
        rem //= e
    if rem != 0:
        raise ValueError("slice id out of range")
    return vals


def n_slices(sliced_labels, extents: dict) -> int:
    n = 1
    for l in sliced_labels:
        n *= extents[l]
    return n


def _extents(tensors, labels) -> dict:
    ext = {}
    for t, lab in zip(tensors, labels):
        if t.ndim != len(lab):
            raise ValueError("tensor rank does not match its label tuple")
        for l, e in zip(lab, t.shape):
            if ext.setdefault(l, e) != e:
                raise ValueError(f"label {l} has inconsistent extents")
    return ext


def _fix(t: np.ndarray, lab: tuple, values: dict):
    """Fix sliced labels of one leaf to their slice values."""
    keep = []
    index = []
    for l in lab:
        if l in values:
            index.append(values[l])
        else:
            index.append(slice(None))
            keep.append(l)
    return np.asarray(t[tuple(index)]), tuple(keep)


def _sum_out(t: np.ndarray, lab: tuple, drop: set):
    axes = tuple(p for p, l in enumerate(lab) if l in drop)
    if axes:
        t = t.sum(axis=axes)
    return t, tuple(l for l in lab if l not in drop)


def pair(A, la, B, lb, keep: set):
    """One pairwise step (Eq. 2.4) with batch labels carried and the rest summed.

    Returns (C, lc) with lc = A's surviving labels followed by B's surviving
    non-shared labels, in their operand order.
    """
    shared = [l for l in la if l in lb]
    only_a = {l for l in la if l not in lb and l not in keep}
    only_b = {l for l in lb if l not in la and l not in keep}
    A, la = _sum_out(A, la, only_a)
    B, lb = _sum_out(B, lb, only_b)
    batch = [l for l in shared if l in keep]
    summed = [l for l in shared if l not in keep]
    free_a = [l for l in la if l not in shared]
    free_b = [l for l in lb if l not in shared]
    out_labels = tuple(batch + free_a + free_b)
    if not batch:
        C = np.tensordot(A, B, axes=([la.index(l) for l in summed],
                                     [lb.index(l) for l in summed]))
        return C, tuple(free_a + free_b)
    # batch labels: one tensordot per batch value, stacked in batch order
    bshape = [A.shape[la.index(l)] for l in batch]
    out = None
    for bv in itertools.product(*[range(e) for e in bshape]):
        ia = [slice(None)] * len(la)
        ib = [slice(None)] * len(lb)
        for l, v in zip(batch, bv):
            ia[la.index(l)] = v
            ib[lb.index(l)] = v
        a_sub, b_sub = A[tuple(ia)], B[tuple(ib)]
        la_sub = [l for l in la if l not in batch]
        lb_sub = [l for l in lb if l not in batch]
        c = np.tensordot(a_sub, b_sub, axes=([la_sub.index(l) for l in summed],
                                             [lb_sub.index(l) for l in summed]))
        if out is None:
            out = np.zeros(tuple(bshape) + c.shape, dtype=np.complex128)
        out[bv] = c
    return out, out_labels


def contract_slice(tensors, labels, open_labels, path, sliced_labels=(), slice_id: int = 0):
    """Amplitudes of one slice, as a flat complex128 vector in open-label order."""
    ext = _extents(tensors, labels)
    open_labels = tuple(open_labels)
    if len(path) != len(tensors) - 1:
        raise ValueError("a pairwise path has n-1 steps")
    values = slice_values(sliced_labels, ext, slice_id) if sliced_labels else {}
    live = {}
    for i, (t, lab) in enumerate(zip(tensors, labels)):
        live[i] = _fix(np.asarray(t, dtype=np.complex128), tuple(lab), values)
    for (i, j) in path:
        (A, la), (B, lb) = live.pop(i), live.pop(j)
        others = set()
        for (_, lo) in live.values():
            others.update(lo)
        keep = set(open_labels) | others
        live[i] = pair(A, la, B, lb, keep)
    (root, lr), = live.values()
    root, lr = _sum_out(root, lr, {l for l in lr if l not in open_labels})
    missing = [l for l in open_labels if l not in lr]
    if missing:
        raise ValueError(f"open labels {missing} are not on any tensor")
    root = np.transpose(root, [lr.index(l) for l in open_labels])
    return np.ascontiguousarray(root).reshape(-1)


def amplitudes(tensors, labels, open_labels, path, sliced_labels=(), slice_ids=None):
    """Sum of slice results in increasing slice-id order (all slices by default)."""
    ext = _extents(tensors, labels)
    if slice_ids is None:
        slice_ids = range(n_slices(sliced_labels, ext)) if sliced_labels else [0]
    acc = None
    for s in slice_ids:
        part = contract_slice(tensors, labels, open_labels, path, sliced_labels, s)
        acc = part if acc is None else acc + part
    return acc


def step_costs(tensors, labels, open_labels, path, sliced_labels=()):
    """Per-step complex GEMM dimensions and the Sec. 2.4 costs of one slice.

    For each step: the batch (B), free-of-A (M), free-of-B (N) and summed (K)
    extents; flops = 8*B*M*N*K (8 real operations per complex multiply-add,
    with each shared batch label counted once); bytes = 8*(|A| + |B| + |C|)
    for complex64 storage.
    """
    ext = _extents(tensors, labels)
    sliced = set(sliced_labels)
    live = {i: tuple(l for l in lab if l not in sliced) for i, lab in enumerate(labels)}
    out = []
    for (i, j) in path:
        la, lb = live.pop(i), live.pop(j)
        others = set()
        for lo in live.values():
            others.update(lo)
        keep = set(open_labels) | others
        prod = lambda ls: int(np.prod([ext[l] for l in ls])) if ls else 1
        batch = [l for l in la if l in lb and l in keep]
        summed = [l for l in la if l in lb and l not in keep]
        trace_a = [l for l in la if l not in lb and l not in keep]
        trace_b = [l for l in lb if l not in la and l not in keep]
        free_a = [l for l in la if l not in lb and l in keep]
        free_b = [l for l in lb if l not in la and l in keep]
        lc = tuple(batch + free_a + free_b)
        B, M, N = prod(batch), prod(free_a), prod(free_b)
        K = prod(summed) * prod(trace_a) * prod(trace_b)
        out.append({"B": B, "M": M, "N": N, "K": K,
                    "flops": 8 * B * M * N * K,
                    "bytes": 8 * (prod(la) + prod(lb) + prod(lc))})
        live[i] = lc
    return out
