"""Contraction paths and slicing for the test and benchmark networks (input generator).

The contraction path is an input of the contraction (Sec. 3.1): a list of N-1
pairs of tensor slots; the result of each pairwise contraction takes the slot
of the first tensor of the pair and the second slot dies.  The paper finds
paths with a simulated-annealing search on contraction trees and chooses the
sliced bonds by dynamic slicing (Sec. 3.2).  This module only needs paths good
enough to drive the tests and benchmarks, so it uses a randomised greedy
search (pick the pair that shrinks memory most, with Gumbel noise, over
several trials) followed by a greedy slicer that cuts, one at a time, the bond
whose removal costs the fewest extra operations until the largest intermediate
fits under the cap (the path is not re-tuned after each cut).

All sizes are tracked as log2 of element counts; extents must be powers of 2.
Operation counts follow Sec. 2.4: 8 real operations per complex multiply-add,
times the product of the extents of every label of the two operands (labels
shared by both operands counted once).
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np


def _log2ext(extents: dict) -> dict:
    out = {}
    for l, e in extents.items():
        b = int(e).bit_length() - 1
        if e < 1 or (1 << b) != e:
            raise ValueError(f"extent {e} of label {l} is not a power of 2")
        out[l] = b
    return out


def replay(labels: list, open_labels, path, sliced=()) -> list:
    """Replay ``path``; returns per-step dicts with the operand and result label sets.

    A label of the two operands is kept in the result when it is open or occurs
    in another live tensor; every other label of the two operands is summed.
    Sliced labels are removed from all tensors first.
    """
    sliced = set(sliced)
    open_set = set(open_labels)
    live = {i: frozenset(l for l in lab if l not in sliced) for i, lab in enumerate(labels)}
    count = defaultdict(int)
    for s in live.values():
        for l in s:
            count[l] += 1
    steps = []
    for (i, j) in path:
        a, b = live.pop(i), live.pop(j)
        for l in a:
            count[l] -= 1
        for l in b:
            count[l] -= 1
        keep = frozenset(l for l in (a | b) if l in open_set or count[l] > 0)
        steps.append({"i": i, "j": j, "a": a, "b": b, "c": keep})
        live[i] = keep
        for l in keep:
            count[l] += 1
    return steps


def path_cost(labels, open_labels, extents, path, sliced=()) -> dict:
    lg = _log2ext(extents)
    steps = replay(labels, open_labels, path, sliced)
    flops = 0.0
    max_log = 0
    for s in steps:
        flops += 8.0 * 2.0 ** sum(lg[l] for l in (s["a"] | s["b"]))
        max_log = max(max_log, sum(lg[l] for l in s["c"]))
    for lab in labels:
        max_log = max(max_log, sum(lg[l] for l in lab if l not in set(sliced)))
    n_slices = 2 ** sum(lg[l] for l in sliced)
    return {"flops_per_slice": flops, "n_slices": n_slices,
            "flops_total": flops * n_slices, "max_log2": max_log}


def greedy_path(labels, open_labels, extents, seed: int = 0, temperature: float = 0.0,
                sliced=(), bitstrings=None) -> list:
    """Randomised greedy pairwise path (memory-reduction score, Gumbel noise).

    With bitstrings (a sparse state, one column per open label), a tensor's open labels
    count as one merged bond over the distinct restrictions of the bitstrings to them
    (Sec. 3.3) instead of 2 per label."""
    rng = np.random.default_rng(seed)
    lg = _log2ext(extents)
    sliced = set(sliced)
    open_set = set(open_labels)
    live = {i: frozenset(l for l in lab if l not in sliced) for i, lab in enumerate(labels)}
    where = defaultdict(set)
    for i, s in live.items():
        for l in s:
            where[l].add(i)
    col = {l: c for c, l in enumerate(open_labels)}
    bkeys = None
    if bitstrings is not None:
        X = np.asarray(bitstrings, dtype=np.uint64)
        bkeys = (X << np.arange(X.shape[1], dtype=np.uint64)).sum(axis=1, dtype=np.uint64)
    distinct = {}

    def size(s):
        if bkeys is None:
            return sum(lg[l] for l in s)
        mask = 0
        closed = 0
        for l in s:
            if l in col:
                mask |= 1 << col[l]
            else:
                closed += lg[l]
        if mask == 0:
            return closed
        if mask not in distinct:
            distinct[mask] = math.log2(len(np.unique(bkeys & np.uint64(mask))))
        return closed + distinct[mask]

    def result(i, j):
        a, b = live[i], live[j]
        return frozenset(l for l in (a | b)
                         if l in open_set or len(where[l] - {i, j}) > 0)

    def score(i, j):
        c = result(i, j)
        return 2.0 ** size(c) - 2.0 ** size(live[i]) - 2.0 ** size(live[j]), c

    def neighbours(i):
        out = set()
        for l in live[i]:
            out |= where[l]
        out.discard(i)
        return out

    cand = {}
    for i in live:
        for j in neighbours(i):
            if i < j:
                cand[(i, j)] = score(i, j)[0]
    path = []
    while len(live) > 1:
        if cand:
            keys = list(cand.keys())
            vals = np.array([cand[k] for k in keys])
            if temperature > 0:
                scale = np.maximum(np.abs(vals), 1.0)
                vals = vals - temperature * scale * np.log(-np.log(rng.uniform(size=len(vals))))
            i, j = keys[int(np.argmin(vals))]
        else:  # disconnected: join the two smallest tensors
            order = sorted(live, key=lambda t: (size(live[t]), t))
            i, j = sorted(order[:2])
        c = result(i, j)
        for t in (i, j):
            for n in neighbours(t):
                cand.pop((min(t, n), max(t, n)), None)
        for l in live[i]:
            where[l].discard(i)
        for l in live[j]:
            where[l].discard(j)
        del live[j]
        live[i] = c
        for l in c:
            where[l].add(i)
        path.append((i, j))
        for n in neighbours(i):
            a, b = min(i, n), max(i, n)
            cand[(a, b)] = score(a, b)[0]
    return path


def _step_masks(labels, open_labels, path):
    """Bitmasks (over label ids) of each step's operand union and result."""
    steps = replay(labels, open_labels, path)
    unions, outs = [], []
    for s in steps:
        unions.append(sum(1 << l for l in (s["a"] | s["b"])))
        outs.append(sum(1 << l for l in s["c"]))
    leaves = [sum(1 << l for l in lab) for lab in labels]
    return unions, outs, leaves


def _masked_log(mask, lg_items):
    if lg_items is None:
        return mask.bit_count()
    return sum(w for l, w in lg_items if (mask >> l) & 1)


def choose_slices(labels, open_labels, extents, path, cap_log2: int, min_sliced: int = 0,
                  max_sliced: int = 64, seed=None, temperature: float = 0.0, start=()) -> list:
    """Greedy slicing: cut bonds until the largest intermediate is <= 2^cap_log2.

    ``start`` are labels already sliced: the result begins with them, in that order, and
    adds bonds after them (with ``max_sliced = len(start) + 1``, exactly one more bond
    unless none is left to cut).

    Slicing a label removes it from every tensor without changing how the other
    labels are classified, so each step's sliced sizes are its unsliced label
    sets minus the sliced labels.  With a seed and temperature > 0 the candidates'
    total costs are multiplied by log-normal noise, giving other slicings of the
    same tree for comparison.
    """
    rng = np.random.default_rng(seed) if (seed is not None and temperature > 0) else None
    lg = _log2ext(extents)
    unit = all(w == 1 for w in lg.values())
    lg_items = None if unit else sorted(lg.items())
    unions, outs, leaves = _step_masks(labels, open_labels, path)
    open_mask = sum(1 << l for l in open_labels)

    def cost(smask):
        keep = ~smask
        flops = sum(2.0 ** _masked_log(u & keep, lg_items) for u in unions)
        mx = max(_masked_log(o & keep, lg_items) for o in outs + leaves)
        return flops * 2.0 ** _masked_log(smask, lg_items), mx

    sliced, smask = list(start), 0
    for l in sliced:
        smask |= 1 << l
    while len(sliced) < max_sliced:
        total, mx = cost(smask)
        if mx <= cap_log2 and len(sliced) >= min_sliced:
            break
        keep = ~smask
        sizes = [_masked_log(o & keep, lg_items) for o in outs]
        big = max(sizes)
        cand_mask = 0
        for o, sz in zip(outs, sizes):
            if mx <= cap_log2 or sz >= big:
                cand_mask |= o
        cand_mask &= ~open_mask & ~smask
        cands = [l for l in range(cand_mask.bit_length()) if (cand_mask >> l) & 1 and lg.get(l, 0) > 0]
        if not cands:
            break
        best = None
        for l in cands:
            t2, m2 = cost(smask | (1 << l))
            if rng is not None:
                t2 *= float(np.exp(temperature * rng.standard_normal()))
            key = (m2 if mx > cap_log2 else 0, t2)
            if best is None or key < best[0]:
                best = (key, l)
        sliced.append(best[1])
        smask |= 1 << best[1]
    return sliced


def find_path(net, cap_log2: int = 60, n_sliced: int = 0, trials: int = 8, seed: int = 0,
              temperature: float = 0.3) -> dict:
    """Best of ``trials`` randomised greedy paths, each sliced to fit ``cap_log2``."""
    extents = net.extents()
    best = None
    for t in range(trials):
        path = greedy_path(net.labels, net.open_labels, extents, seed=seed * 1000 + t,
                           temperature=0.0 if t == 0 else temperature)
        sliced = choose_slices(net.labels, net.open_labels, extents, path, cap_log2,
                               min_sliced=n_sliced, max_sliced=max(n_sliced, 64))
        if n_sliced and len(sliced) != n_sliced:
            continue
        cost = path_cost(net.labels, net.open_labels, extents, path, sliced)
        if cost["max_log2"] > cap_log2:
            continue
        if best is None or cost["flops_total"] < best["cost"]["flops_total"]:
            best = {"path": path, "sliced": sliced, "cost": cost, "trial": t}
    if best is None:
        raise RuntimeError("no path fits the cap with the requested number of sliced labels")
    return best
