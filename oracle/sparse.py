"""CPU complex128 oracle for sparse-state contraction (Sec. 3.3): the amplitudes of a set
of sampled bitstrings from one contraction of the network.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU baseline
leg of the benchmark; never by the GPU product path.

Definition (``definition_amplitudes``).  The network's open labels o_1..o_k are the
output bonds of k measured qubits (extent 2).  For bitstrings x_1..x_S over them, a_s is
the network contracted with every open label fixed to its bit in x_s: one closed
contraction per bitstring, along the same path.

Algorithm (``sparse_state_amplitudes``, Sec. 3.3).  A tensor that holds the open bonds
of a set Q of measured qubits carries, in place of those bonds, one merged bond f whose
values are the distinct restrictions of the bitstrings to Q, in increasing order (a
restriction is the bitstring with the bits outside Q cleared; bit i stands for open
label o_i); a leaf's open bonds become such a bond at once.  When two tensors that both
carry a merged bond meet, the bonds merge: the result's f runs over the distinct
restrictions to Q_A | Q_B, and its slice at a value is the ordinary pairwise product
(Eq. 2.4) of A's slice at the value's restriction to Q_A and B's slice at its
restriction to Q_B -- the concatenation over f of the paper's sparse einsum.  When only
one operand carries a merged bond, f passes through the product as a free index.  The
root's f runs over the distinct bitstrings, and each input bitstring reads its entry.
Slicing (Sec. 3.2) fixes sliced labels per sub-task as in ``contract``; sub-task results
add up in increasing slice id.
"""
from __future__ import annotations

import numpy as np

from . import contract


def bit_keys(bitstrings) -> np.ndarray:
    """uint64 key per bitstring: bit i is the value of open label i."""
    X = np.asarray(bitstrings, dtype=np.uint64)
    if X.ndim != 2 or X.shape[1] > 64:
        raise ValueError("bitstrings must be an (S, k) array with k <= 64")
    if np.any(X > 1):
        raise ValueError("bitstrings hold 0/1 values")
    w = np.left_shift(np.uint64(1), np.arange(X.shape[1], dtype=np.uint64))
    return (X * w).sum(axis=1, dtype=np.uint64)


def definition_amplitudes(tensors, labels, open_labels, path, bitstrings, sliced_labels=()):
    """a_s for each bitstring: the network with its open labels fixed to the bits of x_s."""
    open_pos = {l: i for i, l in enumerate(open_labels)}
    X = np.asarray(bitstrings)
    out = np.zeros(len(X), dtype=np.complex128)
    for s, x in enumerate(X):
        ts, ls = [], []
        for t, lab in zip(tensors, labels):
            idx = tuple(int(x[open_pos[l]]) if l in open_pos else slice(None) for l in lab)
            ts.append(np.asarray(t, dtype=np.complex128)[idx])
            ls.append(tuple(l for l in lab if l not in open_pos))
        out[s] = contract.amplitudes(ts, ls, (), path, sliced_labels)[0]
    return out


def _merged_leaf(t, lab, open_pos, keys_all):
    """A leaf with its open bonds replaced by the merged bond over the restrictions present."""
    q = [open_pos[l] for l in lab if l in open_pos]
    if not q:
        return t, lab, np.uint64(0), None
    mask = np.uint64(sum(1 << i for i in q))
    keys = np.unique(keys_all & mask)
    rest = tuple(l for l in lab if l not in open_pos)
    rows = []
    for key in keys:
        idx = tuple(int((int(key) >> open_pos[l]) & 1) if l in open_pos else slice(None) for l in lab)
        rows.append(t[idx])
    return np.stack(rows), rest, mask, keys


def _step(A, B, keep, keys_all):
    """Pairwise product of two (tensor, labels, mask, keys) operands; f leads when present."""
    (ta, la, ma, ka), (tb, lb, mb, kb) = A, B
    if ka is not None and kb is not None:            # sparse einsum: merge the two bonds
        mask = ma | mb
        keys = np.unique(keys_all & mask)
        ia = np.searchsorted(ka, keys & ma)
        ib = np.searchsorted(kb, keys & mb)
        parts = [contract.pair(ta[i], la, tb[j], lb, keep) for i, j in zip(ia, ib)]
        return np.stack([c for c, _ in parts]), parts[0][1], mask, keys
    if ka is not None:
        parts = [contract.pair(ta[f], la, tb, lb, keep) for f in range(len(ka))]
        return np.stack([c for c, _ in parts]), parts[0][1], ma, ka
    if kb is not None:
        parts = [contract.pair(ta, la, tb[f], lb, keep) for f in range(len(kb))]
        return np.stack([c for c, _ in parts]), parts[0][1], mb, kb
    c, lc = contract.pair(ta, la, tb, lb, keep)
    return c, lc, np.uint64(0), None


def sparse_state_slice(tensors, labels, open_labels, path, bitstrings, sliced_labels=(), slice_id=0):
    """Amplitudes of the bitstrings for one slice, by the sparse-state algorithm."""
    open_pos = {l: i for i, l in enumerate(open_labels)}
    keys_all = bit_keys(bitstrings)
    ext = contract._extents(tensors, labels)
    for l in open_labels:
        if ext.get(l) != 2:
            raise ValueError("open labels of a sparse state are qubit bonds of extent 2")
    values = contract.slice_values(sliced_labels, ext, slice_id) if sliced_labels else {}
    live = {}
    for i, (t, lab) in enumerate(zip(tensors, labels)):
        t, lab = contract._fix(np.asarray(t, dtype=np.complex128), tuple(lab), values)
        live[i] = _merged_leaf(t, lab, open_pos, keys_all)
    for (i, j) in path:
        A, B = live.pop(i), live.pop(j)
        others = set()
        for (_, lo, _, _) in live.values():
            others.update(lo)
        live[i] = _step(A, B, others, keys_all)
    (root, lr, mask, keys), = live.values()
    full = np.uint64((1 << len(open_labels)) - 1) if open_labels else np.uint64(0)
    if mask != full:
        raise ValueError("some open label is on no tensor")
    if keys is None:
        root, lr = contract._sum_out(root, lr, set(lr))
        return np.full(len(keys_all), complex(root))
    root = root.reshape(len(keys), -1).sum(axis=1)   # remaining closed labels (none in a well-formed network)
    return root[np.searchsorted(keys, keys_all)]


def sparse_state_amplitudes(tensors, labels, open_labels, path, bitstrings, sliced_labels=(),
                            slice_ids=None):
    """Sum of slice results in increasing slice-id order (all slices by default)."""
    ext = contract._extents(tensors, labels)
    if slice_ids is None:
        slice_ids = range(contract.n_slices(sliced_labels, ext)) if sliced_labels else [0]
    acc = None
    for s in slice_ids:
        part = sparse_state_slice(tensors, labels, open_labels, path, bitstrings, sliced_labels, s)
        acc = part if acc is None else acc + part
    return acc
