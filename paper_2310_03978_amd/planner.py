"""Contraction-tree refinement by simulated annealing, with dynamic slicing (host-side planning).

Sec. 3.2 scores a contraction tree with log(T_cc + alpha T_mc) + beta log(T_sc): T_cc the
compute cost of all pairwise steps (Eq. for T_cc, Sec. 2.4), T_mc their memory traffic (Eq. for
T_mc), T_sc the size of the largest intermediate; alpha weighs bytes against flops for the
hardware and beta the largest intermediate.  With a `step_time` function (for instance the
learned step-time model, costmodel.StepTimeTable) the first term becomes the log of the summed
predicted step times instead: the hardware weighting is learned rather than a fixed alpha.  Its local update re-pairs the three nearest
descendants of a vertex (for a vertex with children x and y = (a, b): ((x, a), b) or
((x, b), a)), and a sweep visits every vertex from the root towards the leaves.  `refine`
anneals a tree for given sliced labels, keeping every intermediate under a memory cap;
`dynamic_slicing` (Sec. 3.2) cuts one bond at a time with a caller-supplied greedy slicer and
re-anneals the tree after each cut until it fits.

The trees come in and go out as the linear paths that tn_plan_create takes (pair (i, j): the
result takes slot i).  Networks must have every label of extent 2 on exactly two tensors, or on
one if it is open (the tensor networks of qubit circuits); a pairwise step then keeps exactly the
labels of one operand only, so a vertex's label set is the XOR of its children's bitmasks.  Costs
are per slice (sliced labels removed), which for a fixed slicing changes every score by the same
constant.
"""
from __future__ import annotations

import math

import numpy as np
from sortedcontainers import SortedList

from paper_2310_03978_amd import costmodel

# bytes -> flop-equivalents: the split-FP16 MFMA rate (three products) over the HBM bandwidth
DEFAULT_ALPHA = costmodel.PEAK_SPLIT / costmodel.HBM_BW
DEFAULT_BETA = 0.1


class Tree:
    """Binary contraction tree over n leaves; vertex ids: leaves 0..n-1, then internal ones."""

    def __init__(self, labels, open_labels, path, sliced=(), step_time=None):
        self.step_time = step_time
        ids = sorted({l for lab in labels for l in lab})
        self.bit = {l: i for i, l in enumerate(ids)}
        counts = {}
        for lab in labels:
            for l in lab:
                counts[l] = counts.get(l, 0) + 1
        opened = set(open_labels)
        for l, c in counts.items():
            if c != (1 if l in opened else 2):
                raise ValueError("every label must be on two tensors (one if open)")
        self.n = len(labels)
        self.leaf_mask = [self._mask(lab) for lab in labels]
        self.set_sliced(sliced)
        n = self.n
        self.left, self.right, self.parent = {}, {}, {}
        slot = list(range(n))            # slot -> vertex currently stored there
        nxt = n
        for i, j in path:
            v = nxt
            nxt += 1
            self.left[v], self.right[v] = slot[i], slot[j]
            self.parent[slot[i]] = v
            self.parent[slot[j]] = v
            slot[i] = v
            slot[j] = -1
        if nxt != 2 * n - 1:
            raise ValueError("the path must contract all tensors into one")
        self.root = nxt - 1
        self.parent[self.root] = -1
        self._recompute()

    def _mask(self, labs):
        m = 0
        for l in labs:
            m |= 1 << self.bit[l]
        return m

    def set_sliced(self, sliced):
        self.sliced = list(sliced)
        self.keep = ~self._mask(self.sliced)

    # -- costs ---------------------------------------------------------------
    def _size_log(self, m):
        return (m & self.keep).bit_count()

    def _vertex_costs(self, ml, mr):
        """(T_cc, T_mc, log2 size of the result) of one pairwise step, per slice."""
        lu, ll, lr, lc = (self._size_log(ml | mr), self._size_log(ml), self._size_log(mr),
                          self._size_log(ml ^ mr))
        return 8.0 * 2.0 ** lu, 8.0 * (2.0 ** ll + 2.0 ** lr + 2.0 ** lc), lc

    def _vertex_time(self, ml, mr):
        """step_time(m, n, k) of one pairwise step (0 without a step_time function): m, n the
        bits kept from the left and right operand, k the bits they share (summed)."""
        if self.step_time is None:
            return 0.0
        return self.step_time(self._size_log(ml & ~mr), self._size_log(mr & ~ml), self._size_log(ml & mr))

    def _recompute(self):
        self.mask = {v: m for v, m in enumerate(self.leaf_mask)}
        self.cc, self.mc, self.sc, self.tp = {}, {}, {}, {}
        for v in range(self.n, 2 * self.n - 1):   # children have smaller ids than parents
            ml, mr = self.mask[self.left[v]], self.mask[self.right[v]]
            self.mask[v] = ml ^ mr
            self.cc[v], self.mc[v], self.sc[v] = self._vertex_costs(ml, mr)
            self.tp[v] = self._vertex_time(ml, mr)
        self.tcc = sum(self.cc.values())
        self.tmc = sum(self.mc.values())
        self.ttp = sum(self.tp.values())
        self.sizes = SortedList(self.sc.values())
        self.leaf_max = max(self._size_log(m) for m in self.leaf_mask)

    def tsc_log(self):
        return max(self.sizes[-1] if self.sizes else 0, self.leaf_max)

    def score(self, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
        if self.step_time is not None:
            return math.log2(self.ttp) + beta * self.tsc_log()
        return math.log2(self.tcc + alpha * self.tmc) + beta * self.tsc_log()

    # -- local updates ---------------------------------------------------------
    def moves(self, v):
        """Re-pairings at vertex v: (v, c, k) = make (other child of v, child k of c) a new
        vertex and pair it with c's remaining child; c an internal child of v."""
        out = []
        for c in (self.left[v], self.right[v]):
            if c >= self.n:
                out.append((v, c, 0))
                out.append((v, c, 1))
        return out

    def apply(self, v, c, k):
        """Apply a move; returns the undo record.  With x the other child of v and c = (a, b):
        k = 0 pairs (x, a) under c and leaves v = (c, b); k = 1 pairs (x, b), v = (c, a)."""
        x = self.right[v] if self.left[v] == c else self.left[v]
        a, b = self.left[c], self.right[c]
        keep, move = (b, a) if k == 0 else (a, b)     # keep stays under v, move joins x
        old = (self.left[v], self.right[v], self.left[c], self.right[c], self.mask[c],
               self.cc[c], self.mc[c], self.sc[c], self.cc[v], self.mc[v], self.tp[c], self.tp[v])
        self.left[c], self.right[c] = x, move
        self.parent[x] = c
        self.parent[move] = c
        self.left[v], self.right[v] = c, keep
        self.parent[keep] = v
        self.parent[c] = v
        self.tcc -= self.cc[c] + self.cc[v]
        self.tmc -= self.mc[c] + self.mc[v]
        self.ttp -= self.tp[c] + self.tp[v]
        self.sizes.remove(self.sc[c])
        mx, mm = self.mask[x], self.mask[move]
        self.mask[c] = mx ^ mm
        self.cc[c], self.mc[c], self.sc[c] = self._vertex_costs(mx, mm)
        self.cc[v], self.mc[v], _ = self._vertex_costs(self.mask[c], self.mask[keep])
        self.tp[c] = self._vertex_time(mx, mm)
        self.tp[v] = self._vertex_time(self.mask[c], self.mask[keep])
        self.tcc += self.cc[c] + self.cc[v]
        self.tmc += self.mc[c] + self.mc[v]
        self.ttp += self.tp[c] + self.tp[v]
        self.sizes.add(self.sc[c])
        return (v, c, old)

    def undo(self, rec):
        v, c, old = rec
        lv, rv, lc, rc, mcm, ccc, mcc, scc, ccv, mcv, tpc, tpv = old
        self.tcc += ccc + ccv - self.cc[c] - self.cc[v]
        self.tmc += mcc + mcv - self.mc[c] - self.mc[v]
        self.ttp += tpc + tpv - self.tp[c] - self.tp[v]
        self.sizes.remove(self.sc[c])
        self.sizes.add(scc)
        self.left[v], self.right[v], self.left[c], self.right[c] = lv, rv, lc, rc
        for ch in (lv, rv):
            self.parent[ch] = v
        for ch in (lc, rc):
            self.parent[ch] = c
        self.mask[c], self.cc[c], self.mc[c], self.sc[c], self.cc[v], self.mc[v] = mcm, ccc, mcc, scc, ccv, mcv
        self.tp[c], self.tp[v] = tpc, tpv

    # -- paths -------------------------------------------------------------------
    def path(self):
        """The tree as a linear path; a vertex's result takes its left subtree's slot."""
        out = []
        slot = {}

        def visit(v):
            stack = [(v, False)]
            while stack:
                u, done = stack.pop()
                if u < self.n:
                    slot[u] = u
                    continue
                if done:
                    i, j = slot[self.left[u]], slot[self.right[u]]
                    out.append((i, j))
                    slot[u] = i
                else:
                    stack.append((u, True))
                    stack.append((self.right[u], False))
                    stack.append((self.left[u], False))

        visit(self.root)
        return out

    def sweep_order(self):
        """Internal vertices from the root towards the leaves (breadth first)."""
        order, frontier = [], [self.root]
        while frontier:
            nxt = []
            for v in frontier:
                if v >= self.n:
                    order.append(v)
                    nxt += [self.left[v], self.right[v]]
            frontier = nxt
        return order


def anneal_tree(tree, sweeps=40, t_start=1e-4, t_end=1e-7, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA, rng=None,
                cap_log2=None):
    """Metropolis sweeps at temperatures falling geometrically from t_start to t_end (score
    units: log2 of flop-equivalents); moves that would make an intermediate larger than
    2^cap_log2 are rejected.  Returns the best tree seen at the end of a sweep, as a path, and
    its score."""
    rng = rng if rng is not None else np.random.default_rng(0)
    cur = tree.score(alpha, beta)
    best, best_path = cur, tree.path()
    for s in range(sweeps):
        t = t_start * (t_end / t_start) ** (s / max(sweeps - 1, 1))
        for v in tree.sweep_order():
            mv = tree.moves(v)
            if not mv:
                continue
            rec = tree.apply(*mv[int(rng.integers(len(mv)))])
            if cap_log2 is not None and tree.tsc_log() > cap_log2:
                tree.undo(rec)
                continue
            new = tree.score(alpha, beta)
            if new <= cur or rng.random() < math.exp((cur - new) / t):
                cur = new
            else:
                tree.undo(rec)
        if cur < best - 1e-12:
            best, best_path = cur, tree.path()
    return best_path, best


def refine(labels, open_labels, path, sliced=(), cap_log2=None, sweeps=40, t_start=1e-4, t_end=1e-7,
           alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA, seed=0, step_time=None):
    """Anneal the contraction tree of `path` for the given sliced labels; with `cap_log2`, no
    accepted tree has an intermediate above 2^cap_log2 (the input tree must fit).  With
    `step_time(m, n, k)` the score sums predicted step times instead of T_cc + alpha T_mc.

    Returns {"path", "score", "start_score", "tsc_log2", "tcc", "tmc", "time"} (costs per
    slice; "time" is the summed step_time of the result, 0 without one)."""
    tree = Tree(labels, open_labels, path, sliced, step_time)
    if cap_log2 is not None and tree.tsc_log() > cap_log2:
        raise ValueError("the input tree does not fit the cap")
    start = tree.score(alpha, beta)
    p, sc = anneal_tree(tree, sweeps, t_start, t_end, alpha, beta, np.random.default_rng(seed), cap_log2)
    final = Tree(labels, open_labels, p, sliced, step_time)
    return {"path": p, "score": sc, "start_score": start, "tsc_log2": final.tsc_log(), "tcc": final.tcc,
            "tmc": final.tmc, "time": final.ttp}


def dynamic_slicing(labels, open_labels, path, cap_log2, choose, tune_sweeps=30, final_sweeps=200,
                    alpha=DEFAULT_ALPHA, seed=0, step_time=None):
    """Sec. 3.2's dynamic slicing: cut bonds one at a time and re-anneal the tree after each
    cut, until the largest intermediate is at most 2^cap_log2; then anneal under the cap.

    `choose(path, sliced)` returns the labels to slice for the tree of `path`: the list
    `sliced` (the bonds cut so far, kept) followed by one more bond picked greedily for that
    tree.  While the tree does not fit, the annealing weighs the largest intermediate fully
    (beta = 1).  With `step_time` the final annealing under the cap scores trees by summed
    step times (as `refine`).  Raises ValueError when the slicer finds no further bond to cut.
    Returns {"path", "sliced", "score", "tsc_log2", "tcc", "tmc", "time"}."""
    sliced = []
    for it in range(256):
        grown = list(choose(path, list(sliced)))
        if len(grown) != len(sliced) + 1 or grown[:len(sliced)] != sliced:
            raise ValueError("the slicer must keep the bonds cut so far and add exactly one; "
                             f"it returned {len(grown)} labels after {len(sliced)}")
        sliced = grown
        if Tree(labels, open_labels, path, sliced).tsc_log() <= cap_log2:
            break
        path = refine(labels, open_labels, path, sliced, sweeps=tune_sweeps, beta=1.0, alpha=alpha,
                      seed=seed + it)["path"]
        if Tree(labels, open_labels, path, sliced).tsc_log() <= cap_log2:
            break
    else:
        raise ValueError("no slicing of at most 256 bonds fits the cap")
    r = refine(labels, open_labels, path, sliced, cap_log2=cap_log2, sweeps=final_sweeps, alpha=alpha,
               seed=seed + 1000, step_time=step_time)
    r["sliced"] = sliced
    return r


def balanced_step_time(peak=costmodel.PEAK_SPLIT, bandwidth=costmodel.HBM_BW, k_full=6, mn_full=5):
    """Analytic step time with App. A.2's balanced-index feedback, for the annealer when no
    learned model is at hand: the roofline time max(flops / peak, bytes / bandwidth) of a step
    of 2^m x 2^n x 2^k complex extents, divided by an efficiency that halves for every bit k
    falls short of k_full (K below 64: memory latency is not hidden along k) and for every bit
    the smaller of m and n falls short of mn_full (below 32), so the score pushes the tree
    towards contractions whose GEMM extents reach those sizes.  Returns step_time(m, n, k) in
    microseconds."""
    def step_time(m, n, k):
        flops = 8.0 * 2.0 ** (m + n + k)
        nbytes = 8.0 * (2.0 ** (m + k) + 2.0 ** (n + k) + 2.0 ** (m + n))
        eff = 2.0 ** (min(0, k - k_full) + min(0, min(m, n) - mn_full))
        return max(flops / peak, nbytes / bandwidth) / eff * 1e6
    return step_time
