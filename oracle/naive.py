"""Brute-force network contraction by explicit index loops (tiny networks only).

TEST INFRASTRUCTURE ONLY.  Implements the plain definition directly:
a[o] = sum over all assignments of the non-open labels of the product of
every tensor's entry at that assignment.  No pairing, no path, no BLAS: it
cross-checks the label handling (batch, trace, hyperedge labels) of the
pairwise oracle.
"""
from __future__ import annotations

import itertools

import numpy as np


def amplitudes(tensors, labels, open_labels):
    ext = {}
    for t, lab in zip(tensors, labels):
        for l, e in zip(lab, t.shape):
            ext[l] = e
    open_labels = list(open_labels)
    inner = sorted(l for l in ext if l not in open_labels)
    out_shape = [ext[l] for l in open_labels]
    out = np.zeros(int(np.prod(out_shape)) if out_shape else 1, dtype=np.complex128)
    for flat, ovals in enumerate(itertools.product(*[range(e) for e in out_shape])):
        assign = dict(zip(open_labels, ovals))
        total = 0j
        for ivals in itertools.product(*[range(ext[l]) for l in inner]):
            assign.update(zip(inner, ivals))
            term = 1 + 0j
            for t, lab in zip(tensors, labels):
                term *= complex(t[tuple(assign[l] for l in lab)])
                if term == 0:
                    break
            total += term
        out[flat] = total
    return out
