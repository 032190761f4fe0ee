"""Contraction-tree annealing (Sec. 3.2 score and local update), checked against brute force
over every tree of a small network, against the oracle's amplitudes along the refined path,
and for self-consistency of its incremental costs."""
import itertools
import math

import numpy as np
import pytest

from oracle import contract, metrics
from paper_2310_03978_amd import planner
from tn_inputs import configs
from tn_inputs.paths import path_cost


def _tiny_network():
    """Six tensors on a ring with two chords, open labels on tensors 2 and 5 (all extents 2)."""
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (0, 3), (1, 4)]
    labels = [[] for _ in range(6)]
    for e, (a, b) in enumerate(edges):
        labels[a].append(e)
        labels[b].append(e)
    labels[2].append(100)
    labels[5].append(101)
    return labels, [100, 101]


def _all_trees(leaves):
    if len(leaves) == 1:
        yield leaves[0]
        return
    first, rest = leaves[0], leaves[1:]
    for r in range(0, len(rest)):
        for other in itertools.combinations(rest, r):
            left = (first,) + other
            right = tuple(x for x in rest if x not in other)
            for tl in _all_trees(list(left)):
                for tr in _all_trees(list(right)):
                    yield (tl, tr)


def _tree_path(tree):
    out = []

    def go(t):
        if isinstance(t, int):
            return t
        i, j = go(t[0]), go(t[1])
        out.append((i, j))
        return i

    go(tree)
    return out


def test_brute_force_minimum_is_reached():
    labels, opened = _tiny_network()
    trees = list(_all_trees(list(range(6))))
    assert len(trees) == 945                      # (2n - 3)!! unordered binary trees on 6 leaves
    scores = [planner.Tree(labels, opened, _tree_path(t)).score() for t in trees]
    best = min(scores)
    worst_tree = trees[int(np.argmax(scores))]
    found = min(planner.refine(labels, opened, _tree_path(worst_tree), sweeps=300, t_start=1.0, t_end=1e-3,
                               seed=s)["score"] for s in range(4))
    assert found == pytest.approx(best, abs=1e-12)


@pytest.mark.parametrize("workload", ["rqc12", "rqc30"])
def test_tree_round_trip_keeps_costs(workload):
    _, net, best = configs.build(workload)
    t = planner.Tree(net.labels, net.open_labels, best["path"], best["sliced"])
    ref = path_cost(net.labels, net.open_labels, net.extents(), best["path"], best["sliced"])
    assert t.tcc == pytest.approx(ref["flops_per_slice"], rel=1e-12)
    assert t.tsc_log() == ref["max_log2"]
    again = path_cost(net.labels, net.open_labels, net.extents(), t.path(), best["sliced"])
    assert again["flops_per_slice"] == pytest.approx(ref["flops_per_slice"], rel=1e-12)


def test_incremental_costs_match_a_fresh_tree():
    _, net, best = configs.build("rqc30")
    t = planner.Tree(net.labels, net.open_labels, best["path"], best["sliced"])
    rng = np.random.default_rng(3)
    for _ in range(3000):
        order = t.sweep_order()
        mv = t.moves(order[int(rng.integers(len(order)))])
        if not mv:
            continue
        rec = t.apply(*mv[int(rng.integers(len(mv)))])
        if rng.random() < 0.3:
            t.undo(rec)
    fresh = planner.Tree(net.labels, net.open_labels, t.path(), best["sliced"])
    assert t.tcc == pytest.approx(fresh.tcc, rel=1e-9)
    assert t.tmc == pytest.approx(fresh.tmc, rel=1e-9)
    assert t.tsc_log() == fresh.tsc_log()


def test_refined_path_gives_the_same_amplitudes_and_respects_the_cap():
    _, net, best = configs.build("rqc12")
    cap = path_cost(net.labels, net.open_labels, net.extents(), best["path"])["max_log2"]
    r = planner.refine(net.labels, net.open_labels, best["path"], cap_log2=cap, sweeps=20, seed=1)
    assert r["score"] <= r["start_score"] and r["tsc_log2"] <= cap
    a = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    b = contract.amplitudes(net.tensors, net.labels, net.open_labels, r["path"])
    assert metrics.rel_l2(b, a) <= 1e-12
    with pytest.raises(ValueError):
        planner.refine(net.labels, net.open_labels, best["path"], cap_log2=cap - 1)


def test_only_two_tensor_bonds_are_accepted():
    with pytest.raises(ValueError):
        planner.Tree([[0, 1], [0], [0, 1]], [], [(0, 1), (0, 2)])


def test_dynamic_slicing_fits_the_cap_and_keeps_the_amplitudes():
    from tn_inputs.paths import choose_slices
    _, net, best = configs.build("rqc12")
    ext = net.extents()
    cap = path_cost(net.labels, net.open_labels, ext, best["path"])["max_log2"] - 2

    calls = []

    def choose(path, cut):
        calls.append(list(cut))
        return choose_slices(net.labels, net.open_labels, ext, path, cap, start=cut, max_sliced=len(cut) + 1)

    r = planner.dynamic_slicing(net.labels, net.open_labels, best["path"], cap, choose, tune_sweeps=5,
                                final_sweeps=10)
    assert r["tsc_log2"] <= cap and len(r["sliced"]) >= 1
    # one bond per round, the earlier cuts kept
    assert [len(c) for c in calls] == list(range(len(r["sliced"])))
    assert all(r["sliced"][:len(c)] == c for c in calls)
    assert path_cost(net.labels, net.open_labels, ext, r["path"], r["sliced"])["max_log2"] <= cap
    a = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    b = contract.amplitudes(net.tensors, net.labels, net.open_labels, r["path"], r["sliced"])
    assert metrics.rel_l2(b, a) <= 1e-12


def test_dynamic_slicing_raises_when_the_slicer_stops_growing():
    _, net, best = configs.build("rqc12")
    ext = net.extents()
    cap = path_cost(net.labels, net.open_labels, ext, best["path"])["max_log2"] - 2
    with pytest.raises(ValueError, match="exactly one"):
        planner.dynamic_slicing(net.labels, net.open_labels, best["path"], cap, lambda path, cut: list(cut),
                                tune_sweeps=2, final_sweeps=2)


def _analytic_step_time(alpha):
    # T_cc + alpha T_mc of one step from its (m, n, k) bits: the analytic score's own terms
    return lambda m, n, k: 8.0 * 2.0 ** (m + n + k) + alpha * 8.0 * (2.0 ** (m + k) + 2.0 ** (n + k) + 2.0 ** (m + n))


def test_step_time_score_is_kept_incrementally():
    _, net, best = configs.build("rqc12")
    calls = []

    def step_time(m, n, k):
        calls.append((m, n, k))
        return 1.0 + m + 2 * n + 3 * k + (m * n * k) % 5

    tree = planner.Tree(net.labels, net.open_labels, best["path"], step_time=step_time)
    rng = np.random.default_rng(4)
    recs = []
    for _ in range(300):
        v = tree.sweep_order()[int(rng.integers(len(tree.sweep_order())))]
        mv = tree.moves(v)
        if mv:
            recs.append(tree.apply(*mv[int(rng.integers(len(mv)))]))
        if recs and rng.random() < 0.3:
            tree.undo(recs.pop())
    fresh = planner.Tree(net.labels, net.open_labels, tree.path(), step_time=step_time)
    assert tree.ttp == pytest.approx(fresh.ttp, rel=1e-12)
    assert tree.score() == pytest.approx(math.log2(fresh.ttp) + planner.DEFAULT_BETA * fresh.tsc_log(), rel=1e-12)
    assert calls and all(min(c) >= 0 for c in calls)


def test_step_time_score_equal_to_the_analytic_terms_anneals_the_same_way():
    # a step_time that returns exactly T_cc + alpha T_mc of the step makes the learned score
    # the Sec. 3.2 score: the same seed must give the same tree.  alpha is a power of two so
    # that every cost is an exact integer and both sums agree to the last bit.
    _, net, best = configs.build("rqc12")
    alpha = 128.0
    a = planner.refine(net.labels, net.open_labels, best["path"], sweeps=15, seed=3, alpha=alpha)
    b = planner.refine(net.labels, net.open_labels, best["path"], sweeps=15, seed=3,
                       step_time=_analytic_step_time(alpha))
    assert a["path"] != list(best["path"])
    assert a["path"] == b["path"]
    assert a["score"] == b["score"]
    assert b["time"] == a["tcc"] + alpha * a["tmc"]


def test_balanced_step_time_derates_skinny_steps_only():
    """App. A.2: GEMMs with K below 64 or m, n below 32 run below the MFMA rate; the balanced
    step time is the plain roofline time for balanced shapes and larger for skinny ones."""
    f = planner.balanced_step_time(peak=1e15, bandwidth=1e13)

    def roofline(m, n, k):
        return max(8.0 * 2.0 ** (m + n + k) / 1e15,
                   8.0 * (2.0 ** (m + k) + 2.0 ** (n + k) + 2.0 ** (m + n)) / 1e13) * 1e6

    for m, n, k in [(12, 12, 12), (8, 5, 6), (20, 9, 7)]:
        assert f(m, n, k) == pytest.approx(roofline(m, n, k), rel=1e-12)
    # K of 8 (3 bits): 8x the roofline time; n of 2 (1 bit): 16x; both: 128x
    assert f(14, 14, 3) == pytest.approx(8 * roofline(14, 14, 3), rel=1e-12)
    assert f(20, 1, 12) == pytest.approx(16 * roofline(20, 1, 12), rel=1e-12)
    assert f(9, 1, 3) == pytest.approx(128 * roofline(9, 1, 3), rel=1e-12)


def test_balanced_score_anneals_to_a_valid_tree_no_slower_than_the_start():
    """Annealing with the balanced step time keeps the best tree it saw: its summed balanced
    time is at most the starting tree's, and the tree computes the same amplitudes."""
    _, net, best = configs.build("rqc12")
    f = planner.balanced_step_time()
    start = planner.Tree(net.labels, net.open_labels, best["path"], step_time=f).ttp
    b = planner.refine(net.labels, net.open_labels, best["path"], sweeps=20, seed=5, step_time=f)
    assert b["time"] <= start
    a = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    c = contract.amplitudes(net.tensors, net.labels, net.open_labels, b["path"])
    assert metrics.rel_l2(c, a) <= 1e-12
