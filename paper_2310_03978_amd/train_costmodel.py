"""Harvest step timings on this GPU and train the step-time cost model.

    python -m paper_2310_03978_amd.train_costmodel --out paper_2310_03978_amd/data/costmodel_mi355x.json

Data: every step of the plans of seeded uneven lattice circuits (16-28 qubits, depth 8-14),
the 30-qubit 12-cycle workload, a sparse state of that circuit (2048 bitstrings, seed 13), one
slice of the 53-qubit 12-cycle workload (intermediates up to 2^30 elements), the 30-qubit
14-cycle sliced workload (chunks of 8 slices and of 1 slice) and one slice of the 40-qubit
16-cycle workload, in the three precisions, each MFMA step timed with all four tile shapes (HIP
events on the plan's stream).  With `--annealed-workloads`, one slice each of that workload's
tree annealed with the previously shipped model as the score (with and without the floor at the
model's large-step rate) joins the data: the annealer steers toward the step shapes whose speed the
model overstates, and timing them teaches the next model those shapes.  The model is trained on all circuits but the last
`--held-out` ones and the 14-cycle workload; the saved file records the held-out error and
the measured time of the tiles the model picks against the shape heuristic's picks.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2310_03978_amd import costmodel, tn  # noqa: E402
from tn_inputs import configs  # noqa: E402


def log(*a):
    print(*a, flush=True)


def annealed_trees(name: str):
    """The workload's tree (its own sliced bonds and cap) annealed with the shipped model's
    summed step times as the score, without and with the floor at the model's large-step
    rate; [] when no model has been shipped yet."""
    from paper_2310_03978_amd import planner
    if not os.path.exists(costmodel.DEFAULT_MODEL):
        return []
    w = configs.WORKLOADS[name]
    _, net, best = configs.build(name)
    out = []
    with costmodel.CostModel.load() as model:
        table = costmodel.StepTimeTable(model, "f16x3")
        for tag, st in (("learned", table),
                        ("floored", costmodel.StepTimeTable(model, "f16x3", floor_rate=table.large_step_rate()))):
            r = planner.refine(net.labels, net.open_labels, best["path"], best["sliced"], cap_log2=w.cap_log2,
                               sweeps=200, step_time=st)
            out.append((f"{name}{tag}sb1", net, {"path": r["path"], "sliced": list(best["sliced"])}, 1, None))
    return out


def harvest_all(n_circuits: int, precisions, reps: int, extra=(), annealed=()):
    circs = configs.uneven_circuits(n_circuits, seed=5000, cap_log2=25)
    items = [(f"u{i}", net, best, 0, None) for i, (net, best) in enumerate(circs)]
    for name in ["rqc30d12", "rqc30"]:
        _, net, best = configs.build(name)
        items.append((name, net, best, 0, None))
    net, path, bits = configs.sparse_state_workload(count=2048, seed=13)
    items.append(("sparse2048", net, {"path": path}, 0, bits))
    _, net, best = configs.build("rqc53d12")
    items.append(("rqc53d12sb1", net, best, 1, None))
    _, net, best = configs.build("rqc30")
    items.append(("rqc30sb1", net, best, 1, None))
    for name in extra:
        # one slice of a large sliced workload: its largest steps at full size
        _, net, best = configs.build(name)
        items.append((f"{name}sb1", net, best, 1, None))
    for name in annealed:
        items += annealed_trees(name)
    records, defaults = [], {}
    for prec in precisions:
        for tag, net, best, sb, bits in items:
            t0 = time.time()
            with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best.get("sliced", ()),
                         precision=prec, record_steps=True, slice_batch=sb, bitstrings=bits) as p:
                for i, t in enumerate(costmodel.step_tile_ids(p)):
                    defaults[(f"{prec}:{tag}", i)] = t
                recs = costmodel.harvest(p, tag=f"{prec}:{tag}", reps=reps)
            records += recs
            log(f"harvest {prec} {tag}: {len(recs)} records in {time.time() - t0:.1f}s "
                f"(total {len(records)})")
    return records, defaults


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=costmodel.DEFAULT_MODEL)
    ap.add_argument("--records", default=None, help="also write the harvested records (JSON)")
    ap.add_argument("--circuits", type=int, default=160)
    ap.add_argument("--held-out", type=int, default=40)
    ap.add_argument("--extra-workloads", default="rqc40",
                    help="sliced workloads harvested on one slice each (largest steps at full size); the "
                         "53-qubit 14-cycle slicing-choice workload stays out of the data")
    ap.add_argument("--annealed-workloads", default="rqc53d12",
                    help="workloads whose tree, annealed with the shipped model as the score, is "
                         "harvested on one slice")
    ap.add_argument("--precisions", default="f16x3,c64,bf16x3")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        sys.exit("no GPU")
    t0 = time.time()
    extra = [x for x in args.extra_workloads.split(",") if x]
    annealed = [x for x in args.annealed_workloads.split(",") if x]
    records, defaults = harvest_all(args.circuits, args.precisions.split(","), args.reps, extra, annealed)
    if args.records:
        with open(args.records, "w") as f:
            json.dump({"records": records,
                       "defaults": {f"{k[0]}:{k[1]}": v for k, v in defaults.items()}}, f)
    held = {f"u{i}" for i in range(max(0, args.circuits - args.held_out), args.circuits)}
    held |= {"rqc30", "rqc30sb1"}
    train = [r for r in records if r["tag"].split(":")[1] not in held]
    test = [r for r in records if r["tag"].split(":")[1] in held]
    X, us = costmodel.records_to_arrays(train)
    with costmodel.CostModel(seed=args.seed) as m:
        loss = m.fit(X, us, epochs=args.epochs, batch=256, lr=2e-3, seed=args.seed + 1)
        Xt, ust = costmodel.records_to_arrays(test)
        err = m.predict(Xt) - np.log(ust)
        held_rep = costmodel.tile_choice_report(test, m, defaults)
        train_rep = costmodel.tile_choice_report(train, m, defaults)
        meta = {"train_records": len(train), "held_out_records": len(test), "train_mse_ln_us": loss,
                "held_out_rmse_ln_us": float(np.sqrt(np.mean(err ** 2))),
                "held_out_median_abs_rel_err": float(np.median(np.abs(np.expm1(err)))),
                "held_out_tile_choice_us": held_rep, "train_tile_choice_us": train_rep,
                "harvest_and_training_s": round(time.time() - t0, 1),
                "device": torch.cuda.get_device_name(0)}
        m.save(args.out, meta=meta)
    log(json.dumps(meta))


if __name__ == "__main__":
    main()
