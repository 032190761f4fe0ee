#!/usr/bin/env python3
"""Sliced-contraction benchmark on one MI355X.

Workload (default ``rqc30``): the 30-qubit 5x6-lattice random circuit with 14
cycles, 6 open qubits (64 correlated amplitudes) and 8 sliced bonds (256
slices, largest intermediate <= 2^28), on synthetic seeded inputs.  One
benchmark step is one tn_contract_slices call over all 256 slices: the
slice-independent steps, every slice-dependent step of every slice and the
FP64 cross-slice sum.  Inputs are resident on the GPU before timing starts.

Prints ONE JSON line with the split-FP16 throughput as ``value`` (TFLOPS,
algorithmic: 8 real flops per complex multiply-add) and the complex64 run
beside it, the roofline of the dominant kernel (its launches timed with HIP
events on the plan's stream inside the timed region), the batching form
(a slice range of the workload plus uneven 16-28-qubit circuits, plan by plan
against one graph replay) and the CPU oracle timed on one slice of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f16x3": ("mfma", 2500.0, "fp16 MFMA"), "bf16x3": ("mfma", 2500.0, "bf16 MFMA"),
        "c64": ("mfma", 157.3, "fp32 MFMA")}
PRODUCTS = {0: 1, 1: 1, 2: 3, 3: 3}
WAVES = {0: (4, 2), 1: (2, 2), 2: (2, 1), 3: (1, 1)}


def kernel_name(step) -> str:
    """The kernel instance a step launches, as rocprofv3 names it (without arguments)."""
    kind = step["kernel"]
    if kind == 0:
        return "k_gett_small"
    p = kind - 1
    if step.get("lds_copy"):
        return f"void k_gett_dma<{p}, {step['lds_copy'] - 1}>"
    wm, wn = WAVES[step["tile"]]
    return f"void k_gett_mfma<{p}, {wm}, {wn}>"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_precision(tn, torch, net, best, prec, steps, warmup, sample_slice, tuning):
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    plan = tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"],
                   precision=prec, stream=stream, record_steps=True, tuning=tuning)
    plan_s = time.perf_counter() - t0
    info = plan.describe()
    st = plan.steps()
    n_slices = info["n_slices"]
    # sampled slices for the oracle comparison first, so that the launches of the timed
    # passes are the last ones of this plan (a kernel trace can pick them out)
    part = plan.partials(sample_slice)
    for _ in range(warmup):
        plan.contract(0, n_slices)
    torch.cuda.synchronize()
    plan.step_times()          # clear warm-up records
    plan.reset()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        plan.contract(0, n_slices)
    end.record(stream)
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(end) / steps
    step_ms, launches = plan.step_times()
    amps, count = plan.amplitudes()
    assert count == steps * n_slices
    amps = amps / steps
    plan.close()
    flops_step = info["flops_invariant"] + n_slices * info["flops_per_slice"]
    # per kernel kind: total algorithmic flops and measured time in the timed region
    by_kind = {}
    for s, ms, nl in zip(st, step_ms, launches):
        reps = steps * (n_slices if s["per_slice"] else 1)
        d = by_kind.setdefault(kernel_name(s), {"ms": 0.0, "flops": 0.0, "bytes": 0.0, "launches": 0,
                                                "products": PRODUCTS[s["kernel"]]})
        d["ms"] += float(ms)
        d["flops"] += s["flops"] * reps
        d["bytes"] += s["bytes"] * reps
        d["launches"] += int(nl)
    top = sorted(range(len(st)), key=lambda i: -step_ms[i])[:8]
    for i in top:
        s = st[i]
        reps = steps * (n_slices if s["per_slice"] else 1)
        tf = s["flops"] * reps / (step_ms[i] * 1e-3) / 1e12 if step_ms[i] > 0 else 0.0
        log(f"    step {i:3d} {kernel_name(s):28s} tile {s['tile_m']}x{s['tile_n']} "
            f"split {s['split_k']:3d} m={s['m']} n={s['n']} k={s['k']} b={s['batch']} "
            f"{step_ms[i] / steps:8.2f} ms/pass {tf:7.1f} TFLOPS")
    return {"info": info, "ms_per_step": ms_per_step, "flops_step": flops_step, "plan_s": plan_s,
            "tflops": flops_step / (ms_per_step * 1e-3) / 1e12,
            "slices_per_s": n_slices / (ms_per_step * 1e-3),
            "by_kind": by_kind, "amps": amps, "partial": part}


def run_batching(tn, torch, configs, workload, prec, n_small, n_slices, steps):
    """Batching form: a slice range of a large network plus n_small uneven 16-28-qubit
    circuits (every plan with the learned model's tiles), contracted plan by plan
    (tn_contract_slices each) and as one graph replay (tn_group_*); then the large network
    alone, and the small circuits alone plan by plan and as a graph of their own.  Each small
    circuit contracts one slice; its plan is made for chunks of 8 slices (a plan's tiles and K
    splits are chosen for its chunk: for these one-slice contracts chunks of 8 measured
    fastest, 84 ms as a graph against 101 ms with the automatic chunk and 121 ms with 1)."""
    _, net, best = configs.build(workload)
    first = sample_slices(1 << len(best["sliced"]), 1, 404)[0] & ~(n_slices - 1)
    items = [(net, best, first, n_slices)] + [(n, b, 0, 1) for n, b in
                                               configs.uneven_circuits(n_small, seed=1040, cap_log2=22)]
    stream = torch.cuda.current_stream()
    plans = [tn.Plan(n.tensors, n.labels, n.open_labels, b["path"], b.get("sliced", ()),
                     precision=prec, stream=stream, slice_batch=4 if i == 0 else 8, tuning=2)
             for i, (n, b, _, _) in enumerate(items)]
    firsts = [f for _, _, f, _ in items]
    counts = [c for _, _, _, c in items]
    flops = sum(p.describe()["flops_invariant"] + c * p.describe()["flops_per_slice"]
                for p, c in zip(plans, counts))
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()                                   # warm-up (and graph capture)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            fn()
        end.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(end) / steps

    def sequential():
        for p, f, c in zip(plans, firsts, counts):
            p.contract(f, c)

    seq_ms = timed(sequential)
    seq_amps = [p.amplitudes()[0] for p in plans]
    for p in plans:
        p.reset()
    with tn.Group(plans, stream=stream) as g:
        grp_ms = timed(lambda: g.contract(firsts, counts))
        info = g.describe()
        grp_amps = [p.amplitudes()[0] for p in plans]
    same = all(np.array_equal(a, b) for a, b in zip(seq_amps, grp_amps))
    # where the graph's gain comes from: the large network alone, and the uneven circuits
    # alone plan by plan and as their own graph
    big_ms = timed(lambda: plans[0].contract(firsts[0], counts[0]))

    def small_sequential():
        for p in plans[1:]:
            p.contract(0, 1)

    for p in plans[1:]:
        p.reset()
    small_seq_ms = timed(small_sequential)
    small_amps = [p.amplitudes()[0] for p in plans[1:]]
    for p in plans[1:]:
        p.reset()
    with tn.Group(plans[1:], stream=stream) as g:
        small_grp_ms = timed(lambda: g.contract([0] * (len(plans) - 1), [1] * (len(plans) - 1)))
        small_same = all(np.array_equal(a, p.amplitudes()[0]) for a, p in zip(small_amps, plans[1:]))
    for p in plans:
        p.close()
    return {"workload": workload, "plans": len(plans), "workload_slices": [first, first + n_slices],
            "small_circuits": n_small, "flops": flops, "sequential_ms": round(seq_ms, 3),
            "graph_ms": round(grp_ms, 3), "speedup": round(seq_ms / grp_ms, 3),
            "graph_tflops": round(flops / (grp_ms * 1e-3) / 1e12, 3),
            "graph_kernels": info["n_kernels"], "graph_branches": info["n_branches"],
            "amplitudes_identical": bool(same), "precision": prec,
            "large_network_alone_ms": round(big_ms, 3),
            "small_circuits_alone": {"sequential_ms": round(small_seq_ms, 3), "graph_ms": round(small_grp_ms, 3),
                                     "speedup": round(small_seq_ms / small_grp_ms, 3),
                                     "amplitudes_identical": bool(small_same)}}


def run_batching_full(tn, torch, configs, prec, n_slices, per_graph, n_small):
    """The batching form at its stated size: n_slices slices of the 40-qubit 5x8 16-cycle network
    (the tree of Sec. 3.2's dynamic slicing under the 2^28 cap, slice ranges aligned to the chunk
    size) plus n_small uneven 16-28-qubit circuits contracted in full (every slice of each, sliced
    to a 2^24 cap), every plan with the learned model's tiles.  Contracted plan by plan
    (tn_contract_slices per plan, the large range in pieces of per_graph slices), then through one
    group whose graphs each carry per_graph of the large network's slices and a share of every
    small circuit's slices (each circuit's slices cut into as many contiguous pieces as there are
    graphs, piece p of circuit j in graph (p + j) mod graphs): captured beforehand
    (tn_group_prepare, timed on the host) and replayed (timed with events).  Amplitudes and slice
    counts of every plan compared bit for bit."""
    from paper_2310_03978_amd import planner
    from tn_inputs.paths import choose_slices
    _, net, best = configs.build("rqc40")
    w = configs.WORKLOADS["rqc40"]
    ext = net.extents()
    t0 = time.perf_counter()
    dyn = planner.dynamic_slicing(
        net.labels, net.open_labels, best["path"], w.cap_log2,
        lambda pth, cut: choose_slices(net.labels, net.open_labels, ext, pth, w.cap_log2, start=cut,
                                       max_sliced=len(cut) + 1))
    planning_s = time.perf_counter() - t0
    n_total = 1 << len(dyn["sliced"])
    sb = 16
    first = sample_slices(n_total, 1, 404)[0] & ~(n_slices - 1)
    if first + n_slices > n_total:
        first = n_total - n_slices
    pieces = [(first + o, per_graph) for o in range(0, n_slices, per_graph)]
    G = len(pieces)
    log(f"  rqc40 tree: {len(dyn['sliced'])} sliced bonds ({n_total} slices), planned in {planning_s:.1f}s; "
        f"slices [{first}, {first + n_slices}) in {G} graphs of {per_graph}")
    smalls = configs.uneven_circuits(n_small, seed=1040, cap_log2=24)
    stream = torch.cuda.current_stream()
    plans = [tn.Plan(net.tensors, net.labels, net.open_labels, dyn["path"], dyn["sliced"], precision=prec,
                     stream=stream, slice_batch=sb, tuning=2)]
    plans += [tn.Plan(n.tensors, n.labels, n.open_labels, b["path"], b.get("sliced", ()), precision=prec,
                      stream=stream, slice_batch=1, tuning=2) for n, b in smalls]
    small_counts = [p.describe()["n_slices"] for p in plans[1:]]
    info0 = plans[0].describe()
    flops = n_slices * info0["flops_per_slice"] + info0["flops_invariant"] + sum(
        p.describe()["flops_invariant"] + c * p.describe()["flops_per_slice"] for p, c in zip(plans[1:], small_counts))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # plan by plan
    torch.cuda.synchronize()
    ev0.record(stream)
    for p, c in zip(plans[1:], small_counts):
        p.contract(0, c)
    for i, (f, c) in enumerate(pieces):
        plans[0].contract(f, c)
        ev1.record(stream)
        torch.cuda.synchronize()
        if (i + 1) % max(1, G // 8) == 0 or i + 1 == G:
            log(f"  plan by plan: {f + c - first} of {n_slices} slices done, {ev0.elapsed_time(ev1) / 1e3:.1f}s")
    seq_ms = ev0.elapsed_time(ev1)
    seq_amps = [p.amplitudes()[0] for p in plans]
    for p in plans:
        p.reset()

    def small_piece(j, i):
        q = (i - j) % G                       # piece q of circuit j goes to graph i
        n = small_counts[j]
        lo, hi = q * n // G, (q + 1) * n // G
        return lo, hi - lo

    ranges = []
    for i, (f, c) in enumerate(pieces):
        sp = [small_piece(j, i) for j in range(n_small)]
        ranges.append(([f] + [x[0] for x in sp], [c] + [x[1] for x in sp]))
    assert all(sum(r[1][1 + j] for r in ranges) == small_counts[j] for j in range(n_small))
    with tn.Group(plans, stream=stream) as g:
        t0 = time.perf_counter()
        kernels, branches = [], []
        for i, (fr, cr) in enumerate(ranges):
            g.prepare(fr, cr)
            kernels.append(g.describe()["n_kernels"])
            branches.append(g.describe()["n_branches"])
            if (i + 1) % max(1, G // 8) == 0:
                log(f"  captured {i + 1} of {G} graphs, {time.perf_counter() - t0:.1f}s")
        capture_s = time.perf_counter() - t0
        torch.cuda.synchronize()
        ev0.record(stream)
        for i, (fr, cr) in enumerate(ranges):
            g.contract(fr, cr)
            if (i + 1) % max(1, G // 8) == 0 or i + 1 == G:
                ev1.record(stream)
                torch.cuda.synchronize()
                log(f"  graph replays: {i + 1} of {G} done, {ev0.elapsed_time(ev1) / 1e3:.1f}s")
        grp_ms = ev0.elapsed_time(ev1)
        grp_amps = [p.amplitudes() for p in plans]
    same = all(np.array_equal(a, b[0]) for a, b in zip(seq_amps, grp_amps))
    counts_ok = grp_amps[0][1] == n_slices and all(b[1] == c for b, c in zip(grp_amps[1:], small_counts))
    for p in plans:
        p.close()
    return {"workload": "rqc40: 40-qubit 5x8 lattice, 16 cycles, 6 open qubits, cap 2^28, dynamic slicing",
            "precision": prec, "sliced_labels": len(dyn["sliced"]), "workload_slices": [first, first + n_slices],
            "slices": n_slices, "slices_per_graph": per_graph, "graphs": G, "small_circuits": n_small,
            "small_circuit_slices": int(sum(small_counts)), "planning_s": round(planning_s, 1), "flops": flops,
            "sequential_ms": round(seq_ms, 1), "graph_ms": round(grp_ms, 1), "speedup": round(seq_ms / grp_ms, 3),
            "graph_tflops": round(flops / (grp_ms * 1e-3) / 1e12, 2),
            "graph_slices_per_s": round(n_slices / (grp_ms * 1e-3), 2),
            "capture_s": round(capture_s, 2), "graph_kernels_max": max(kernels), "graph_kernels_total": sum(kernels),
            "graph_branches_max": max(branches), "amplitudes_identical": bool(same and counts_ok)}


def run_tuning_modes(tn, torch, net, best, prec, n_slices):
    """Whole-plan time over n_slices slices with tiles from the shape heuristic, the learned
    step-time model and measured autotuning."""
    stream = torch.cuda.current_stream()
    out = {}
    for name, tuning in (("heuristic", 0), ("learned_model", 2), ("autotune", 1)):
        t0 = time.perf_counter()
        with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"],
                     precision=prec, stream=stream, tuning=tuning) as p:
            plan_s = time.perf_counter() - t0
            p.contract(0, 8)
            torch.cuda.synchronize()
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            s.record(stream)
            p.contract(0, n_slices)
            e.record(stream)
            torch.cuda.synchronize()
            out[name] = {"ms": round(s.elapsed_time(e), 3), "plan_s": round(plan_s, 3)}
            p.amplitudes()
    out["slices"] = n_slices
    out["precision"] = prec
    out["learned_vs_heuristic_speedup"] = round(out["heuristic"]["ms"] / out["learned_model"]["ms"], 3)
    return out


COUNTERS = os.path.join(ROOT, "profiles", "gett_rqc30_counters.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2310_03978_amd", "csrc", "tn_kernels.hip")


def measured_traffic(kernel: str, slice_batch: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when there is none for it, the kernel source changed since the counters were taken (the
    summary records the SHA-256 of tn_kernels.hip it was measured with) or the plan's slice
    chunk differs from the one the counters were taken with (the launches would differ)."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if f"kernel source sha256: {src}" not in text or f"slice chunk: {slice_batch}\n" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic per launch:") and f"`{kernel}`" in line:
            return float(line.rsplit(" ", 2)[-2])
    return None


def run_mixed_precision(tn, torch, net, best, prec, sample_ids, n_slices, budgets):
    """Per-step precision (Sec. 4.3, Table 3): single products on the top k split steps of
    the library's ranking by measured time, three products elsewhere.  For each k: time of
    n_slices slices and the partial amplitudes of the sampled slices (compared with the
    oracle afterwards).  Then, for each epsilon_L2^2 budget, the library's own choice of k
    (tn_plan_choose_single_products on the sampled slices, against its three-product
    amplitudes) with the time of the chosen plan."""
    stream = torch.cuda.current_stream()
    out, chosen = [], []

    def timed(p):
        p.contract(0, min(8, n_slices))
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        e0 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        p.contract(0, n_slices)
        e0.record(stream)
        torch.cuda.synchronize()
        p.reset()
        return s0.elapsed_time(e0)

    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"],
                 precision=prec, stream=stream, tuning=2) as p:
        order = p.rank_split_steps(by_time=True)
        n_split = len(order)
        ks = sorted({0, 1, 2, 4, 8, 16, n_split} & set(range(n_split + 1)))
        st = p.steps()
        n_all = p.describe()["n_slices"]
        total = sum(s["flops"] * (n_all if s["per_slice"] else 1) for s in st if s["kernel"] in (2, 3))
        for k in ks:
            top = p.single_product_top(k)
            share = sum(st[i]["flops"] * (n_all if st[i]["per_slice"] else 1) for i in top) / max(total, 1.0)
            ms = timed(p)
            out.append({"k": k, "split_flops_share": round(share, 4), "ms": round(ms, 3),
                        "partial": p.partials(sample_ids)})
        for budget in budgets:
            t0 = time.perf_counter()
            k, eps = p.choose_single_products(budget, sample_ids)
            choose_s = time.perf_counter() - t0
            ms = timed(p)
            chosen.append({"budget": budget, "k": k, "eps_l2sq_vs_three_products": eps, "ms": round(ms, 3),
                           "choose_s": round(choose_s, 2), "partial": p.partials(sample_ids)})
    return out, chosen


def rel_l2(got, ref):
    """||got - ref|| / ||ref|| over all entries (GPU-against-GPU comparisons of the bench)."""
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def max_err(got, ref):
    """max |got - ref| / max |ref| over all entries."""
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def run_precision_form(tn, torch, configs, n_timed, n_check):
    """The precision form at its own size (53-qubit 6x9-minus-one lattice, 12 cycles, 512
    correlated amplitudes, largest intermediate 2^30): split FP16, split BF16 and complex64
    on the same slices.  Timing: n_timed consecutive slices from a seeded position (every
    slice costs the same).  Errors: the split precisions' partial amplitudes of n_check
    seeded slices (seed 303) against complex64's (no oracle slice of this network finishes
    in minutes).  Also returns the amplitudes of the 30-qubit 12-cycle sub-case in every
    precision, which the CPU leg compares with the oracle's stored amplitudes."""
    _, net, best = configs.build("rqc53d12")
    n_slices = 1 << len(best["sliced"])
    check = sample_slices(n_slices, n_check, 303)
    first = sample_slices(n_slices, 1, 304)[0] & ~(n_timed - 1)
    stream = torch.cuda.current_stream()
    out = {"workload": configs.WORKLOADS["rqc53d12"].description, "slices_timed": n_timed,
           "timed_range": [first, first + n_timed], "checked_slices": check, "n_slices": n_slices}
    parts = {}
    for prec in ("f16x3", "bf16x3", "c64"):
        t0 = time.perf_counter()
        with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"], precision=prec,
                     stream=stream, tuning=2) as p:
            plan_s = time.perf_counter() - t0
            info = p.describe()
            parts[prec] = p.partials(check)
            p.contract(first, min(n_timed, 2))   # warm-up
            torch.cuda.synchronize()
            p.reset()
            s0 = torch.cuda.Event(enable_timing=True)
            e0 = torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            p.contract(first, n_timed)
            e0.record(stream)
            torch.cuda.synchronize()
            ms = s0.elapsed_time(e0)
        flops = info["flops_per_slice"] * n_timed + info["flops_invariant"]
        out[prec] = {"ms_per_slice": round(ms / n_timed, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
                     "slices_per_s": round(n_timed / (ms * 1e-3), 3), "plan_s": round(plan_s, 2)}
        log(f"  precision form {prec}: {out[prec]}")
    out["flops_per_slice"] = info["flops_per_slice"]
    out["max_intermediate"] = info["max_intermediate"]
    for prec in ("f16x3", "bf16x3"):
        out[prec]["rel_l2_vs_c64"] = rel_l2(parts[prec], parts["c64"])
        out[prec]["speedup_vs_c64"] = round(out["c64"]["ms_per_slice"] / out[prec]["ms_per_slice"], 3)
    _, snet, sbest = configs.build("rqc30d12")
    sub_amps = {}
    for prec in ("f16x3", "bf16x3", "c64"):
        with tn.Plan(snet.tensors, snet.labels, snet.open_labels, sbest["path"], precision=prec,
                     stream=stream) as p:
            p.contract()
            sub_amps[prec], _ = p.amplitudes()
    return out, sub_amps


def precision_subcase_vs_oracle(configs, sub_amps):
    """CPU leg: the 30-qubit 12-cycle sub-case's amplitudes in every precision against the
    oracle's stored amplitudes (tests/golden fixture, checked to belong to this network)."""
    import importlib.util
    from oracle import metrics
    path = os.path.join(ROOT, "tests", "golden", "make_rqc30d12_amplitudes.py")
    spec = importlib.util.spec_from_file_location("make_rqc30d12_amplitudes", path)
    fx = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fx)
    digest, ref = fx.read_fixture()
    _, snet, sbest = configs.build("rqc30d12")
    sub = {"workload": configs.WORKLOADS["rqc30d12"].description,
           "fixture_matches_network": digest == fx.network_digest(snet, sbest)}
    for prec, amps in sub_amps.items():
        sub[prec] = {k: float(v) for k, v in metrics.report(amps, ref).items()}
    return sub


def run_precision_form_full(tn, torch, configs, prec, n_slices, piece=128):
    """The precision form's evaluation at its stated size: n_slices consecutive slices of the
    53-qubit 12-cycle network (512 correlated amplitudes, largest intermediate 2^30) summed
    into one FP64 accumulator in one precision, timed with HIP events from the first piece's
    launch to the last one's end.  Pieces of `piece` slices are enqueued one ahead of the
    one being waited for, so the device never idles on the host's progress lines.  The same
    two seeded slices as the default precision-form record (seed 303) are compared with
    complex64, and the accumulated amplitudes are summarised (squared norm, largest)."""
    _, net, best = configs.build("rqc53d12")
    total = 1 << len(best["sliced"])
    first = sample_slices(total, 1, 304)[0] & ~(n_slices - 1)
    check = sample_slices(total, 2, 303)
    stream = torch.cuda.current_stream()
    out = {"workload": configs.WORKLOADS["rqc53d12"].description, "precision": prec,
           "slices": n_slices, "range": [first, first + n_slices], "n_slices": total}
    parts = {}
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"], precision="c64",
                 stream=stream, tuning=2) as p:
        parts["c64"] = p.partials(check)
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"], precision=prec,
                 stream=stream, tuning=2) as p:
        info = p.describe()
        parts[prec] = p.partials(check)
        p.contract(first, 2)   # warm-up
        torch.cuda.synchronize()
        p.reset()
        n_pieces = (n_slices + piece - 1) // piece
        ends = []
        start = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        t0 = time.perf_counter()
        for i in range(n_pieces + 1):
            if i < n_pieces:
                p.contract(first + i * piece, min(piece, n_slices - i * piece))
                e = torch.cuda.Event(enable_timing=True)
                e.record(stream)
                ends.append(e)
            if i >= 1:
                ends[i - 1].synchronize()
                done = min(i * piece, n_slices)
                log(f"  precision form {prec}: {done}/{n_slices} slices, {time.perf_counter() - t0:.0f} s")
        ms = start.elapsed_time(ends[-1])
        amps, count = p.amplitudes()
    flops = info["flops_per_slice"] * n_slices + info["flops_invariant"]
    out.update({"ms": round(ms, 1), "ms_per_slice": round(ms / n_slices, 3),
                "tflops": round(flops / (ms * 1e-3) / 1e12, 2), "slices_per_s": round(n_slices / (ms * 1e-3), 3),
                "flops": flops, "slices_accumulated": int(count), "amplitudes": int(len(amps)),
                "sum_abs2": float(np.sum(np.abs(amps) ** 2)), "max_abs": float(np.max(np.abs(amps))),
                "checked_slices": check, "rel_l2_vs_c64_checked": rel_l2(parts[prec], parts["c64"]),
                "max_err_vs_c64_checked": max_err(parts[prec], parts["c64"])})
    return out


def run_operand_data_check(tn, torch, net, best, desc, n_slices=64, reps=3):
    """The headline plan (split FP16, shape-heuristic tiles so that every variant runs the
    same launches) contracted over the same slices with the circuit's own leaves, with
    leaves of constant value (every multiplier input repeats: the least switching) and with
    seeded Gaussian leaves: time of the LDS-copy steps and of all steps per pass (HIP
    events per launch).  The instruction stream is the same in all three, so a difference
    in time is the clock the chip holds under each data's power draw."""
    rng = np.random.default_rng(5)
    variants = [("circuit", net.tensors), ("constant", [np.ones_like(t) for t in net.tensors]),
                ("gaussian", [(rng.standard_normal(t.shape) + 1j * rng.standard_normal(t.shape)).astype(t.dtype)
                              for t in net.tensors]), ("circuit_again", net.tensors)]
    out = {"workload": desc, "precision": "f16x3", "slices_per_pass": n_slices, "passes": reps}
    for name, tensors in variants:
        with tn.Plan(tensors, net.labels, net.open_labels, best["path"], best["sliced"], precision="f16x3",
                     record_steps=True, tuning=0) as p:
            st = p.steps()
            dma = [i for i, s in enumerate(st) if s["lds_copy"] == 1]
            p.contract(0, 16)
            torch.cuda.synchronize()
            p.step_times()
            p.reset()
            copy_ms, all_ms = [], []
            for _ in range(reps):
                p.contract(0, n_slices)
                torch.cuda.synchronize()
                ms, _ = p.step_times()
                copy_ms.append(float(sum(ms[i] for i in dma)))
                all_ms.append(float(ms.sum()))
            amps, _ = p.amplitudes()
        out[name] = {"lds_copy_steps_ms": round(float(np.median(copy_ms)), 2),
                     "all_steps_ms": round(float(np.median(all_ms)), 2),
                     "finite": bool(np.all(np.isfinite(amps)))}
        log(f"  operand data {name}: {out[name]}")
    out["constant_speedup_of_copy_steps"] = round(out["circuit"]["lds_copy_steps_ms"] /
                                                  out["constant"]["lds_copy_steps_ms"], 3)
    return out


def run_sparse_state(tn, torch, configs, reps):
    """Sparse-state contraction (Sec. 3.3): amplitudes of 4096 sampled bitstrings of the
    30-qubit 12-cycle circuit with every qubit measured, in one contraction; split FP16
    timed, complex64 for the speed ratio and the amplitude agreement.  Returns the record
    and the amplitudes of both precisions (per bitstring)."""
    net, path, bits = configs.sparse_state_workload()
    stream = torch.cuda.current_stream()
    out = {"workload": "rqc30d12 circuit, all 30 qubits measured, 4096 uniform bitstrings, unsliced",
           "bitstrings": int(len(bits))}
    amps = {}
    for prec in ("f16x3", "c64"):
        with tn.Plan(net.tensors, net.labels, net.open_labels, path, precision=prec, stream=stream,
                     bitstrings=bits, record_steps=True, tuning=2) as p:
            info = p.describe()
            st = p.steps()
            flops = info["flops_invariant"] + info["flops_per_slice"]
            p.contract()
            torch.cuda.synchronize()
            p.step_times()
            p.reset()
            n = reps if prec == "f16x3" else 1
            s0 = torch.cuda.Event(enable_timing=True)
            e0 = torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            for _ in range(n):
                p.contract()
            e0.record(stream)
            torch.cuda.synchronize()
            ms = s0.elapsed_time(e0) / n
            step_ms, _ = p.step_times()
            a, c = p.amplitudes()
            amps[prec] = a / c
            merged_ms = sum(float(m) for m, s in zip(step_ms, st) if s["merged_bits"] >= 0)
            out[prec] = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
                         "bitstrings_per_s": round(len(bits) / (ms * 1e-3), 1),
                         "sparse_einsum_time_share": round(merged_ms / max(float(step_ms.sum()), 1e-9), 4)}
            out["flops"] = flops
            out["sparse_einsum_flops_share"] = round(sum(s["flops"] for s in st if s["merged_bits"] >= 0) / flops, 4)
            out["max_intermediate"] = info["max_intermediate"]
    out["speedup_vs_c64"] = round(out["c64"]["ms"] / out["f16x3"]["ms"], 3)
    out["rel_l2_f16x3_vs_c64"] = float(np.linalg.norm(amps["f16x3"] - amps["c64"]) / np.linalg.norm(amps["c64"]))
    return out, amps


def sparse_state_vs_oracle(configs, amps, n):
    """CPU leg: the oracle's definition of n seeded bitstrings' amplitudes of the sparse-state
    workload (one closed complex128 contraction per bitstring, along a greedy path of the
    closed network), against the GPU amplitudes of both precisions."""
    from oracle import metrics, sparse
    from tn_inputs.paths import greedy_path, path_cost
    net, _, bits = configs.sparse_state_workload()
    ids = sample_slices(len(bits), n, 707)
    opened = set(net.open_labels)
    closed = [tuple(l for l in lab if l not in opened) for lab in net.labels]
    ext = net.extents()
    cands = [greedy_path(closed, (), ext, seed=k, temperature=0.0 if k == 0 else 0.3) for k in range(6)]
    cpath = min(cands, key=lambda p: path_cost(closed, (), ext, p)["flops_total"])
    t0 = time.perf_counter()
    ref = sparse.definition_amplitudes(net.tensors, net.labels, net.open_labels, cpath, bits[ids])
    out = {"bitstrings": ids, "oracle_s": round(time.perf_counter() - t0, 1)}
    for prec, a in amps.items():
        got = a[ids]
        out[prec] = {"rel_l2": metrics.rel_l2(got, ref), "max_err": metrics.max_err(got, ref)}
    return out


def run_permute(tn, torch, reps):
    """HBM bandwidth of the LDS-staged permutation kernel (Sec. 2.4 transposes) on 2^28
    complex64 elements (2 GiB read, 2 GiB written): a plain copy, a 2-D transpose, a rank-5
    transpose and a random permutation of 28 bits; bytes = 16 per element.  Each call is
    timed with HIP events on the stream it runs on (descriptor upload + kernel), median of
    reps calls; torch's own device copy of the same bytes is timed the same way."""
    n_bits = 28
    x = torch.randn(1 << n_bits, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    rng = np.random.default_rng(11)
    cases = {"copy": ([1 << 14, 1 << 14], [0, 1]), "transpose_2d": ([1 << 14, 1 << 14], [1, 0]),
             "transpose_rank5": ([64, 64, 64, 32, 32], [3, 0, 4, 2, 1]),
             "random_bit_permutation": ([2] * n_bits, [int(v) for v in rng.permutation(n_bits)])}
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()                                   # warm-up
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    out = {}
    for name, (shape, perm) in cases.items():
        xs = x.view(*shape)
        ms = timed(lambda: tn.tn_permute(xs, perm, y, stream))
        gbs = 16.0 * (1 << n_bits) / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 3), "GB/s": round(gbs, 1), "frac_of_8TB/s": round(gbs / 8000.0, 3)}
    ms = timed(lambda: y.copy_(x))
    out["torch_copy_reference"] = {"ms": round(ms, 3), "GB/s": round(16.0 * (1 << n_bits) / (ms * 1e-3) / 1e9, 1)}
    del x, y
    return out


def run_harvest_check(tn, torch, configs):
    """The step timings the learned cost model trains on, aggregated per kernel instance:
    one harvest-style pass of the 30-qubit 12-cycle workload in split FP16 (every MFMA step
    with each of the four tile ids: one warm-up contraction, then two recorded), timed with
    HIP events on the plan's stream around each launch (tn_plan_step_times).  Run under
    rocprofv3 --kernel-trace, the per-dispatch durations of the same kernels can be
    compared with these means.  Split-K steps are counted but left out of the means (their
    recorded time includes the reduction launch)."""
    _, net, best = configs.build("rqc30d12")
    agg = {}
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"], precision="f16x3",
                 record_steps=True, tuning=0) as p:
        mfma = [i for i, s in enumerate(p.steps()) if s["kernel"] != 0]
        for tile in range(4):
            for i in mfma:
                p.set_tile(i, tile)
            steps = p.steps()
            p.contract(0, 1)
            p.step_times()
            for _ in range(2):
                p.contract(0, 1)
            ms, cnt = p.step_times()
            for i in mfma:
                if cnt[i] == 0:
                    continue
                a = agg.setdefault(kernel_name(steps[i]), {"launches": 0, "ms": 0.0, "split_k_launches": 0})
                if steps[i]["split_k"] > 1:
                    a["split_k_launches"] += int(cnt[i])
                    continue
                a["launches"] += int(cnt[i])
                a["ms"] += float(ms[i])
        torch.cuda.synchronize()
    return {k: {"launches": v["launches"], "split_k_launches": v["split_k_launches"],
                "mean_us": round(1e3 * v["ms"] / v["launches"], 3) if v["launches"] else None}
            for k, v in sorted(agg.items())}


def sample_slices(n_slices: int, count: int, seed: int = 137):
    """Seeded sample of distinct slice ids (sorted)."""
    rng = np.random.default_rng(seed)
    return sorted(int(x) for x in rng.choice(n_slices, size=min(count, n_slices), replace=False))


def run_slicing_choice(tn, torch, configs, workload, prec, n_candidates, n_timed):
    """Slicings of the workload's contraction tree (the greedy slicer, and the slicer with
    noisy costs for further candidates, each cutting bonds until the cap holds) ranked for
    the whole job (all slices) three ways: by flops (T_cc), by the analytic flop/byte
    roofline and by the learned model's predicted time with its own tiles.  Every
    candidate is then timed on the GPU (n_timed seeded slices at full size, the model's
    tiles) and its time extrapolated to all its slices (slices cost the same), so each
    ranking's pick and its rank agreement with the measurement can be compared.  Seven more
    candidates: the greedy slicing on the tree refined by the annealer (Sec. 3.2 score and
    local updates, every intermediate kept under the cap), Sec. 3.2's dynamic slicing (one
    bond at a time, the tree re-annealed after each cut), the same two with the learned
    model's summed step times as the annealing score in place of T_cc + alpha T_mc, the same
    two with every predicted step time held to at least its flops at the model's own large-step
    rate, and the annealer scored by App. A.2's balanced-index step time, timed the same way."""
    from paper_2310_03978_amd import costmodel, planner
    from tn_inputs.paths import choose_slices
    _, net, best = configs.build(workload)
    w = configs.WORKLOADS[workload]
    ext = net.extents()
    cands, seen = [], set()
    for t in range(n_candidates):
        sliced = list(best["sliced"]) if t == 0 else choose_slices(
            net.labels, net.open_labels, ext, best["path"], w.cap_log2, seed=t, temperature=0.5)
        if tuple(sorted(sliced)) not in seen:
            seen.add(tuple(sorted(sliced)))
            cands.append((best["path"], sliced))
    t0 = time.perf_counter()
    ref = planner.refine(net.labels, net.open_labels, best["path"], best["sliced"], cap_log2=w.cap_log2, sweeps=200)
    anneal_s = time.perf_counter() - t0
    cands.append((ref["path"], list(best["sliced"])))
    t0 = time.perf_counter()
    dyn = planner.dynamic_slicing(
        net.labels, net.open_labels, best["path"], w.cap_log2,
        lambda pth, cut: choose_slices(net.labels, net.open_labels, ext, pth, w.cap_log2, start=cut,
                                       max_sliced=len(cut) + 1))
    dyn_s = time.perf_counter() - t0
    cands.append((dyn["path"], dyn["sliced"]))
    stream = torch.cuda.current_stream()
    rows = []
    with costmodel.CostModel.load() as model:
        # the same two refinements scored by the learned model (summed predicted step times
        # in place of T_cc + alpha T_mc)
        table = costmodel.StepTimeTable(model, prec)
        t0 = time.perf_counter()
        lref = planner.refine(net.labels, net.open_labels, best["path"], best["sliced"], cap_log2=w.cap_log2,
                              sweeps=200, step_time=table)
        lanneal_s = time.perf_counter() - t0
        cands.append((lref["path"], list(best["sliced"])))
        t0 = time.perf_counter()
        ldyn = planner.dynamic_slicing(
            net.labels, net.open_labels, best["path"], w.cap_log2,
            lambda pth, cut: choose_slices(net.labels, net.open_labels, ext, pth, w.cap_log2, start=cut,
                                           max_sliced=len(cut) + 1), step_time=table)
        ldyn_s = time.perf_counter() - t0
        cands.append((ldyn["path"], ldyn["sliced"]))
        # the learned score with every step held to at most the model's own large-step rate
        floored = costmodel.StepTimeTable(model, prec, floor_rate=table.large_step_rate())
        fref = planner.refine(net.labels, net.open_labels, best["path"], best["sliced"], cap_log2=w.cap_log2,
                              sweeps=200, step_time=floored)
        cands.append((fref["path"], list(best["sliced"])))
        fdyn = planner.dynamic_slicing(
            net.labels, net.open_labels, best["path"], w.cap_log2,
            lambda pth, cut: choose_slices(net.labels, net.open_labels, ext, pth, w.cap_log2, start=cut,
                                           max_sliced=len(cut) + 1), step_time=floored)
        cands.append((fdyn["path"], fdyn["sliced"]))
        # App. A.2's balanced-index feedback in analytic form (no model)
        bref = planner.refine(net.labels, net.open_labels, best["path"], best["sliced"], cap_log2=w.cap_log2,
                              sweeps=200, step_time=planner.balanced_step_time())
        cands.append((bref["path"], list(best["sliced"])))
        for path, sliced in cands:
            args = (net.tensors, net.labels, net.open_labels, path, sliced)
            with tn.Plan(*args, precision=prec, host_only=True, slice_batch=1) as h:
                info = h.describe()
                r = {"sliced_labels": len(sliced), "n_slices": info["n_slices"],
                     "flops": info["flops_invariant"] + info["n_slices"] * info["flops_per_slice"],
                     "analytic_s": costmodel.analytic_plan_us(h) / 1e6,
                     "predicted_s": costmodel.predict_plan_us(h, model) / 1e6}
            with tn.Plan(*args, precision=prec, stream=stream, tuning=2, slice_batch=1) as p:
                ids = sample_slices(info["n_slices"], n_timed + 1, 505)
                p.contract(ids[0], 1)
                torch.cuda.synchronize()
                s0 = torch.cuda.Event(enable_timing=True)
                e0 = torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                for sid in ids[1:]:
                    p.contract(sid, 1)
                e0.record(stream)
                torch.cuda.synchronize()
                p.amplitudes()
                r["measured_ms_per_slice"] = s0.elapsed_time(e0) / n_timed
            r["measured_s"] = r["measured_ms_per_slice"] * r["n_slices"] / 1e3
            rows.append(r)

    def ranks(v):
        order = sorted(range(len(v)), key=lambda i: v[i])
        out = [0] * len(v)
        for k, i in enumerate(order):
            out[i] = k
        return out

    def spearman(x, y):
        rx, ry = ranks(x), ranks(y)
        n = len(x)
        return 1.0 - 6.0 * sum((a - b) ** 2 for a, b in zip(rx, ry)) / (n * (n * n - 1)) if n > 1 else 1.0

    meas = [r["measured_s"] for r in rows]
    out = {"workload": f"{workload}: {w.description}", "cap_log2": w.cap_log2, "candidates": len(rows),
           "slices_timed_per_candidate": n_timed, "precision": prec,
           "fastest_measured_s": round(min(meas), 1)}
    for name, key in (("flops", "flops"), ("analytic", "analytic_s"), ("learned_model", "predicted_s")):
        vals = [r[key] for r in rows]
        i = min(range(len(rows)), key=lambda j: vals[j])
        out[f"pick_by_{name}"] = {"candidate": i, "sliced_labels": rows[i]["sliced_labels"],
                                  "measured_s": round(rows[i]["measured_s"], 1),
                                  "rank_correlation_with_measured": round(spearman(vals, meas), 3)}
    for name, key in (("analytic", "analytic_s"), ("learned_model", "predicted_s")):
        errs = sorted(abs(r[key] / r["measured_s"] - 1.0) for r in rows)
        out[f"pick_by_{name}"]["median_abs_rel_error_of_job_time"] = round(errs[len(errs) // 2], 3)
    out["learned_vs_flops_speedup"] = round(out["pick_by_flops"]["measured_s"] /
                                            out["pick_by_learned_model"]["measured_s"], 3)
    out["learned_vs_analytic_speedup"] = round(out["pick_by_analytic"]["measured_s"] /
                                               out["pick_by_learned_model"]["measured_s"], 3)
    ia, idy, ila, ild, ifa, ifd, ib = (len(rows) - 7, len(rows) - 6, len(rows) - 5, len(rows) - 4,
                                       len(rows) - 3, len(rows) - 2, len(rows) - 1)
    out["annealed_tree"] = {"candidate": ia, "sliced_labels": rows[ia]["sliced_labels"],
                            "score_before": round(ref["start_score"], 4), "score_after": round(ref["score"], 4),
                            "flops_vs_greedy_tree": round(rows[ia]["flops"] / rows[0]["flops"], 4),
                            "measured_speedup_vs_greedy_tree": round(rows[0]["measured_s"] / rows[ia]["measured_s"], 3),
                            "anneal_s": round(anneal_s, 2)}
    out["dynamic_slicing"] = {"candidate": idy, "sliced_labels": rows[idy]["sliced_labels"],
                              "flops_vs_greedy_tree": round(rows[idy]["flops"] / rows[0]["flops"], 4),
                              "measured_speedup_vs_greedy_tree": round(rows[0]["measured_s"] / rows[idy]["measured_s"], 3),
                              "planning_s": round(dyn_s, 1)}
    # the learned model as the annealing score, against the analytic score on the same task
    out["learned_score"] = {
        "annealed_tree": {"candidate": ila, "sliced_labels": rows[ila]["sliced_labels"],
                          "flops_vs_analytic_annealed": round(rows[ila]["flops"] / rows[ia]["flops"], 4),
                          "measured_speedup_vs_analytic_annealed": round(rows[ia]["measured_s"] / rows[ila]["measured_s"], 3),
                          "predicted_step_us_per_slice": round(lref["time"], 1), "anneal_s": round(lanneal_s, 2)},
        "dynamic_slicing": {"candidate": ild, "sliced_labels": rows[ild]["sliced_labels"],
                            "flops_vs_analytic_dynamic": round(rows[ild]["flops"] / rows[idy]["flops"], 4),
                            "measured_speedup_vs_analytic_dynamic": round(rows[idy]["measured_s"] / rows[ild]["measured_s"], 3),
                            "measured_speedup_vs_greedy_tree": round(rows[0]["measured_s"] / rows[ild]["measured_s"], 3),
                            "planning_s": round(ldyn_s, 1)},
        "table_entries": len(table.cache),
        "floored": {"floor_tflops": round(floored.floor_rate / 1e12, 1),
                    "annealed_tree": {"candidate": ifa, "flops_vs_analytic_annealed": round(rows[ifa]["flops"] / rows[ia]["flops"], 4),
                                      "measured_speedup_vs_analytic_annealed": round(rows[ia]["measured_s"] / rows[ifa]["measured_s"], 3)},
                    "dynamic_slicing": {"candidate": ifd, "sliced_labels": rows[ifd]["sliced_labels"],
                                        "flops_vs_analytic_dynamic": round(rows[ifd]["flops"] / rows[idy]["flops"], 4),
                                        "measured_speedup_vs_analytic_dynamic": round(rows[idy]["measured_s"] / rows[ifd]["measured_s"], 3)}}}
    out["balanced_score"] = {"candidate": ib, "sliced_labels": rows[ib]["sliced_labels"],
                             "flops_vs_analytic_annealed": round(rows[ib]["flops"] / rows[ia]["flops"], 4),
                             "measured_speedup_vs_analytic_annealed": round(rows[ia]["measured_s"] / rows[ib]["measured_s"], 3)}
    out["rows"] = [{k: (round(v, 3) if isinstance(v, float) and k != "flops" else v) for k, v in r.items()}
                   for r in rows]
    return out


def cpu_baseline(net, best, ids, flops_slice):
    """The complex128 oracle on the host cores over the sampled slices: (partials, record)."""
    from oracle import contract
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        blas = [x.get("num_threads", 0) for x in threadpool_info() if x.get("user_api") == "blas"]
        if blas:
            threads = max(blas)
    except Exception:
        pass
    blas_threads = threads
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    t0 = time.perf_counter()
    refs = [contract.contract_slice(net.tensors, net.labels, net.open_labels, best["path"],
                                    best["sliced"], sid) for sid in ids]
    dt = time.perf_counter() - t0
    n = len(ids)
    return np.asarray(refs), {
        "value": flops_slice * n / dt / 1e12, "unit": "TFLOPS", "cores": threads, "kind": "oracle",
        "os_cpu_count": os.cpu_count(), "blas_threads": blas_threads, "cpu_model": model,
        "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
        "slices_per_s": n / dt, "seconds": dt,
        "sample": f"{n} slices (seeded ids {ids}) of the same workload, complex128 numpy "
                  f"tensordot along the same path; flops counted as for the GPU"}


def counter_run(tn, torch, net, best, precs, tuning):
    """One pass over all slices per precision, with the tiles of the timed run, plus a
    plain copy of known size.

    Meant to run under rocprofv3 --pmc: the pass has the launch mix of one timed pass
    (its launches are the last of the plan; autotuning launches come first), and the
    copy (an identity permutation of 2^26 complex64 = 512 MiB read and 512 MiB
    written) calibrates FETCH_SIZE and WRITE_SIZE against known byte counts.
    """
    stream = torch.cuda.current_stream()
    for prec in precs:
        with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"],
                     precision=prec, stream=stream, tuning=tuning) as plan:
            info = plan.describe()
            plan.contract(0, info["n_slices"])
            plan.amplitudes()
            log(f"counter run {prec}: one pass over {info['n_slices']} slices")
    n = 1 << 26
    x = torch.zeros(n, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    tn.tn_permute(x.view(1 << 13, 1 << 13), [0, 1], y)
    torch.cuda.synchronize()
    log(f"calibration copy: {n * 8} bytes read, {n * 8} bytes written")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rqc30")
    ap.add_argument("--precisions", default="f16x3,c64")
    ap.add_argument("--extra-precisions", default="bf16x3",
                    help="more precisions on the same workload, timed with steps // 4 (at least 1)")
    ap.add_argument("--precision-form-slices", type=int, default=8,
                    help="timed slices per precision of the 53-qubit 12-cycle precision form (0 = skip)")
    ap.add_argument("--cpu-slices", type=int, default=8,
                    help="slices in the CPU oracle sample (and in the per-slice error check)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", type=int, default=1, help="1 = autotune tile shapes at plan creation")
    ap.add_argument("--no-tuning-modes", dest="tuning_modes", action="store_false",
                    help="skip the heuristic / learned-model / autotune comparison")
    ap.add_argument("--slicing-candidates", type=int, default=8,
                    help="candidate trees for the slicing choice: flops vs analytic vs learned model (0 = skip)")
    ap.add_argument("--slicing-workload", default="rqc53d14")
    ap.add_argument("--batching", type=int, default=256,
                    help="uneven circuits in the batching-form measurement (0 = skip it)")
    ap.add_argument("--batching-workload", default="rqc40")
    ap.add_argument("--batching-slices", type=int, default=32)
    ap.add_argument("--batching-full", default="",
                    help="only the batching form at full size, PREC:SLICES:PER_GRAPH (e.g. f16x3:4096:2048)")
    ap.add_argument("--precision-form-full", default="",
                    help="PREC:SLICES: only the precision form's evaluation of SLICES slices of the "
                         "53-qubit 12-cycle network in one precision")
    ap.add_argument("--operand-data-check", action="store_true",
                    help="only the headline plan's step times on the circuit's leaves, constant leaves "
                         "and Gaussian leaves (one JSON line)")
    ap.add_argument("--no-permute", dest="permute", action="store_false",
                    help="skip the permutation-kernel bandwidth measurement")
    ap.add_argument("--permute-only", action="store_true",
                    help="only the permutation-kernel bandwidth measurement (one JSON line)")
    ap.add_argument("--harvest-check", action="store_true",
                    help="only the cost model's event-timed step means per kernel (one JSON line)")
    ap.add_argument("--no-sparse-state", dest="sparse_state", action="store_false",
                    help="skip the sparse-state (sampled bitstrings) measurement")
    ap.add_argument("--no-mixed-precision", dest="mixed_precision", action="store_false",
                    help="skip the per-step precision (single products on the costliest steps) sweep")
    ap.add_argument("--counter-run", action="store_true",
                    help="one pass per precision and a calibration copy, for rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: slices are independent sub-tasks and the "
              "multi-GPU sum of partial amplitudes is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_2310_03978_amd import tn
    from tn_inputs import configs
    if args.permute_only:
        print(json.dumps({"permute": run_permute(tn, torch, max(args.steps, 5))}), flush=True)
        return
    if args.harvest_check:
        print(json.dumps({"harvest_check": run_harvest_check(tn, torch, configs)}), flush=True)
        return
    if args.precision_form_full:
        prec, n = args.precision_form_full.split(":")
        log(f"precision form at full size: {prec}, {n} slices of rqc53d12")
        print(json.dumps({"precision_form_full": run_precision_form_full(tn, torch, configs, prec, int(n))}),
              flush=True)
        return
    if args.batching_full:
        prec, n, per = args.batching_full.split(":")
        log(f"batching form at full size: {prec}, {n} slices of rqc40 + {args.batching} uneven circuits")
        print(json.dumps({"batching_full": run_batching_full(tn, torch, configs, prec, int(n), int(per),
                                                             args.batching)}), flush=True)
        return

    t0 = time.perf_counter()
    circ, net, best = configs.build(args.workload)
    w = configs.WORKLOADS[args.workload]
    log(f"workload {args.workload}: {w.description}; path found in {time.perf_counter() - t0:.1f}s")
    precs = [p for p in args.precisions.split(",") if p]
    if args.operand_data_check:
        print(json.dumps({"operand_data_check": run_operand_data_check(tn, torch, net, best, f"{args.workload}: {w.description}")}), flush=True)
        return
    if args.counter_run:
        counter_run(tn, torch, net, best, precs, args.tuning)
        return
    n_slices_total = 1
    for lab in best["sliced"]:
        n_slices_total *= net.extents()[lab]
    sample_ids = sample_slices(n_slices_total, args.cpu_slices)
    runs = {}
    for prec in precs:
        log(f"running {prec}: warmup {args.warmup}, steps {args.steps}")
        runs[prec] = run_precision(tn, torch, net, best, prec, args.steps, args.warmup,
                                   sample_ids, args.tuning)
        r = runs[prec]
        log(f"  {prec}: {r['ms_per_step']:.1f} ms/step, {r['tflops']:.1f} TFLOPS, "
            f"{r['slices_per_s']:.1f} slices/s")
    for prec in [p for p in args.extra_precisions.split(",") if p and p not in runs]:
        k = max(1, args.steps // 4)
        log(f"running {prec}: warmup 1, steps {k}")
        runs[prec] = run_precision(tn, torch, net, best, prec, k, 1, sample_ids, args.tuning)
        runs[prec]["steps"] = k
        r = runs[prec]
        log(f"  {prec}: {r['ms_per_step']:.1f} ms/step, {r['tflops']:.1f} TFLOPS, "
            f"{r['slices_per_s']:.1f} slices/s")
    head = precs[0]
    main_run = runs[head]
    info = main_run["info"]

    # roofline of the dominant kernel (most measured time) of the headline run
    kinds = main_run["by_kind"]
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    dk = kinds[dom]
    achieved = dk["flops"] / (dk["ms"] * 1e-3) / 1e12
    bound, peak, peak_name = PEAK[head] if dom != "k_gett_small" else ("alu", 157.3, "fp32 vector")
    roof = {"bound": bound, "kernel": dom, "achieved": round(achieved, 2),
            "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(dom, info["slice_batch"]),
            "launches": dk["launches"], "avg_launch_ms": round(dk["ms"] / max(dk["launches"], 1), 4),
            "flops_per_launch": dk["flops"] / max(dk["launches"], 1),
            "algorithmic_bytes_per_launch": dk["bytes"] / max(dk["launches"], 1),
            "time_share": round(dk["ms"] / sum(v["ms"] for v in kinds.values()), 4),
            "peak_dtype": peak_name}
    if dk["products"] > 1:
        roof["executed_mfma_tflops"] = round(achieved * dk["products"], 2)
        roof["executed_frac"] = round(achieved * dk["products"] / peak, 4)

    out = {"metric": "sliced-contraction TFLOPS & slices/s, FP16-scaled vs complex64, <=1e-3 amp err",
           "value": round(main_run["tflops"], 3), "unit": "TFLOPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(main_run["ms_per_step"], 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": head, "data": "synthetic",
           "config": {"workload": f"{args.workload}: {w.description}",
                      "n_slices": info["n_slices"], "n_amplitudes": info["n_amplitudes"],
                      "flops_per_step": main_run["flops_step"],
                      "max_intermediate": info["max_intermediate"],
                      "slice_batch": info["slice_batch"], "precision": head},
           "slices_per_s": round(main_run["slices_per_s"], 2)}
    for prec, r in runs.items():
        out[prec] = {"tflops": round(r["tflops"], 3), "slices_per_s": round(r["slices_per_s"], 2),
                     "ms_per_step": round(r["ms_per_step"], 3),
                     "plan_and_tuning_s": round(r["plan_s"], 3), "steps": r.get("steps", args.steps)}
        if prec != "c64" and "c64" in runs:
            out[prec]["speedup_vs_c64"] = round(runs["c64"]["ms_per_step"] / r["ms_per_step"], 3)
    if "c64" in runs and head != "c64":
        out["speedup_vs_c64"] = round(runs["c64"]["ms_per_step"] / main_run["ms_per_step"], 3)
        ref_c64 = runs["c64"]["amps"]
        out["rel_l2_vs_c64_full"] = float(np.linalg.norm(main_run["amps"] - ref_c64) / np.linalg.norm(ref_c64))
    out["roofline"] = roof
    if args.tuning_modes:
        log("tile choice: shape heuristic vs learned model vs autotune on 32 slices")
        out["tile_choice"] = run_tuning_modes(tn, torch, net, best, head, 32)
        log(f"  {out['tile_choice']}")
    if args.slicing_candidates > 0:
        log(f"slicing choice on {args.slicing_workload}: {args.slicing_candidates} candidate trees, "
            f"flops vs analytic model vs learned model")
        out["slicing_choice"] = run_slicing_choice(tn, torch, configs, args.slicing_workload, head,
                                                   args.slicing_candidates, 2)
        log(f"  {out['slicing_choice']}")
    if args.permute:
        log("permutation kernel bandwidth: 2^28 complex64")
        out["permute"] = run_permute(tn, torch, 5)
        log(f"  {out['permute']}")
    if args.sparse_state:
        log("sparse-state contraction: 4096 bitstrings of the 30-qubit 12-cycle circuit")
        out["sparse_state"], sparse_amps = run_sparse_state(tn, torch, configs, 2)
        log(f"  {out['sparse_state']}")
    mixed = None
    if args.mixed_precision and head != "c64":
        log(f"per-step precision: single products on the top-k split steps, {head}")
        mixed = run_mixed_precision(tn, torch, net, best, head, sample_ids, 32, (1e-5, 1e-4))
    if args.precision_form_slices > 0:
        log(f"precision form: rqc53d12, {args.precision_form_slices} timed slices per precision")
        out["precision_form"], subcase_amps = run_precision_form(tn, torch, configs,
                                                                 args.precision_form_slices, 2)
    if args.batching > 0:
        log(f"batching form: {args.batching} uneven circuits + {args.batching_slices} slices of "
            f"{args.batching_workload}")
        out["batching"] = run_batching(tn, torch, configs, args.batching_workload, head, args.batching,
                                       args.batching_slices, 2)
        log(f"  {out['batching']}")
    if not args.no_cpu_baseline:
        from oracle import metrics
        ref, cb = cpu_baseline(net, best, sample_ids,
                               info["flops_per_slice"] + info["flops_invariant"])
        out["cpu_baseline"] = cb
        if args.precision_form_slices > 0:
            out["precision_form"]["oracle_subcase_30q"] = precision_subcase_vs_oracle(configs, subcase_amps)
        if args.sparse_state:
            log("sparse state: 4 sampled bitstrings against the oracle's definition (CPU)")
            out["sparse_state"]["vs_oracle_bitstrings"] = sparse_state_vs_oracle(configs, sparse_amps, 4)
        if mixed:
            # Table 3's trend: time and error against the oracle as single products spread
            top, chosen = mixed
            base_ms = top[0]["ms"]
            out["mixed_precision"] = {
                "precision": head, "slices_timed": 32, "sampled_slices": len(ref), "ranking": "measured time",
                "top_k": [{"k": r["k"], "split_flops_share": r["split_flops_share"], "ms": r["ms"],
                           "eps_l2sq": metrics.eps_l2sq(r["partial"], ref), "rel_l2": metrics.rel_l2(r["partial"], ref)}
                          for r in top],
                "budget_choice": [{"budget": c["budget"], "k": c["k"],
                                   "eps_l2sq_vs_three_products": c["eps_l2sq_vs_three_products"],
                                   "eps_l2sq_vs_oracle": metrics.eps_l2sq(c["partial"], ref),
                                   "rel_l2_vs_oracle": metrics.rel_l2(c["partial"], ref), "ms": c["ms"],
                                   "speedup_vs_three_products": round(base_ms / c["ms"], 3),
                                   "choose_s": c["choose_s"]} for c in chosen]}
            log(f"  {out['mixed_precision']}")
        for prec, r in runs.items():
            # errors of the sampled slices' amplitudes against the complex128 oracle
            per = [metrics.rel_l2(a, b) for a, b in zip(r["partial"], ref)]
            out[prec]["vs_oracle_slices"] = {
                "slices": len(per), "rel_l2": metrics.rel_l2(r["partial"], ref),
                "rel_l2_max_slice": max(per), "eps_l2sq": metrics.eps_l2sq(r["partial"], ref),
                "fidelity": metrics.fidelity(r["partial"], ref)}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
