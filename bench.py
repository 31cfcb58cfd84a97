"""Benchmark: search nodes/s and constraint revisions/s on one MI355X.

Workload (the random binary CSP configuration): the model-RB style instance
with n=40 variables, domain size 16, 25% of the variable pairs constrained
(195 tables) and 90 of the 256 value pairs of each table forbidden
(tightness 0.35), base seed 2, index 0, counted exhaustively; plus 13-queens
counted exhaustively (73,712 solutions) as the second check of the same
configuration.

The RB instance has ~2e11 solutions, so the bench counts it in its 16
top-level slices: slice v is the sub-CSP with x0 restricted to value v.
First-fail branches on x0 at the root of the full instance (all domains have
16 values; lowest index wins), so the 16 slices are exactly the 16 subtrees
of the root: their counts sum to the full count and their node counts sum to
the full node count minus the root.  One step = one slice (slices taken in
order 0, 1, ... from the first timed step; warmup steps use slices from the
top, 15, 14, ...) plus one 13-queens count.  --steps 16 covers the whole
instance once.

The JSON line reports nodes/s (value), revisions/s, the roofline of the
search kernel (algorithmic domain/table/trail bytes over the kernel time
measured with HIP events on the library's stream), the learned-vs-first-fail
leg (untimed: a policy trained on the plain solver's sibling subtree sizes
at nodes of --learned-train seeded instances, then time-to-all-solutions and
node counts of --learned-eval held-out instances under both orderings), and
the CPU oracle timed on a bounded sample of the RB workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1909_09213_amd/csrc/cubics_search.hip",
                  "paper_1909_09213_amd/csrc/cubics_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_kernel_rb_traffic.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def rb_instance():
    import cspgen
    return cspgen.rb(0, n=40, d=16, dens_pm=250, tight_pm=350, base=cspgen.SEED_RB)


def rb_slice(inst, v):
    return inst.fix({0: v})


def traffic_per_launch(launches):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(budget_s: float):
    """The oracle (single thread) counting seeded sub-CSPs of the same RB
    instance: x0..x4 fixed to seeded values, until ~budget_s of CPU time."""
    import numpy as np

    import oracle
    inst = rb_instance()
    rng = np.random.default_rng(20240)
    nodes = revs = 0
    t_used = 0.0
    k = 0
    while t_used < budget_s and k < 400:
        vals = rng.integers(0, 16, 5)
        sub = inst.fix({i: int(v) for i, v in enumerate(vals)})
        t0 = time.perf_counter()
        r = oracle.solve(sub, oracle.MODE_COUNT)
        t_used += time.perf_counter() - t0
        nodes += r.nodes
        revs += r.revisions
        k += 1
    return {"value": nodes / t_used, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "revisions_per_s": revs / t_used,
            "sample": f"oracle counting {k} seeded sub-CSPs of the RB instance "
                      f"(x0..x4 fixed to seeded values): {nodes} nodes in {t_used:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--layout", type=int, default=0, help="0 auto, 1 lane, 2 seg")
    ap.add_argument("--split", type=int, default=0, help="eager split target (0 = donation only)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--learned-train", type=int, default=4000,
                    help="training instances of the learned-vs-first-fail leg (0 = skip it)")
    ap.add_argument("--learned-eval", type=int, default=1024)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 256 MiB device-to-device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; --gpus must be 1 (sharding a "
              "search over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.steps + args.warmup > 16:
        print("bench.py: need 1 <= steps and steps + warmup <= 16 (the instance has 16 slices)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import cspgen
    from paper_1909_09213_amd import cubics as cb

    ctx = cb.Context(0)
    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    inst = rb_instance()
    q13 = ctx.load(cspgen.queens(13))
    slices = {v: ctx.load(rb_slice(inst, v)) for v in range(16)}

    # the library's autotuner picks the revision layout for each shape (untimed)
    tuned = {}
    # windows long enough that start-up and drain do not decide the choice
    for name, p, t in (("rb", slices[15], 1500), ("queens13", q13, 100)):
        chosen, div, rates = ctx.autotune([p], cb.MODE_COUNT, time_ms=t, rates=True)
        names = {1: "lane", 2: "seg", 3: "var"}
        tuned[name] = {"chosen": names[chosen], "worker_divisor": div,
                       "nodes_per_ms": {f"{names[k]}/{d}": round(v) for (k, d), v in rates.items()}}

    def step(v):
        r1 = ctx.solve(slices[v], cb.MODE_COUNT, layout=args.layout, split_target=args.split)
        r2 = ctx.solve(q13, cb.MODE_COUNT, layout=args.layout, split_target=args.split)
        return r1, r2

    for w in range(args.warmup):
        step(15 - w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb_res, q_res = [], []
    for s in range(args.steps):
        r1, r2 = step(s)
        rb_res.append(r1)
        q_res.append(r2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    for r in q_res:
        assert r.count == 73712, f"13-queens count {r.count} != 73712"
    nodes = sum(r.nodes for r in rb_res) + sum(r.nodes for r in q_res)
    revs = sum(r.revisions for r in rb_res) + sum(r.revisions for r in q_res)
    # the dominant kernel: the search kernel's RB-slice launches of the timed
    # region (13-queens takes ~0.1% of the time, in its own autotuned variant)
    launches = len(rb_res)
    bytes_per_launch = sum(r.alg_bytes for r in rb_res) / launches
    ms_per_launch = sum(r.kernel_ms for r in rb_res) / launches
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    traffic = traffic_per_launch(launches)
    out = {
        "metric": "search nodes/s + revisions/s at 1 GPU; time-to-all-solutions learned vs first-fail",
        "value": nodes / dt,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "model-RB random binary CSP n=40 d=16 density 0.25 tightness 0.35 "
                               "(195 tables, 90/256 pairs forbidden, seed 2 index 0) count-all in "
                               "16 x0-slices, + 13-queens count-all",
                   "slices_timed": list(range(args.steps)),
                   "layout": args.layout, "split_target": args.split,
                   "autotuned_layout": tuned},
        "revisions_per_s": revs / dt,
        "solutions": {"rb_slices": [r.count for r in rb_res], "queens13": q_res[0].count},
        "nodes": {"rb_slices": [r.nodes for r in rb_res], "queens13": q_res[0].nodes},
        "kernel_ms": {"rb_slices": [round(r.kernel_ms, 3) for r in rb_res],
                      "queens13": [round(r.kernel_ms, 3) for r in q_res]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "search_kernel, RB-slice launches of the timed steps "
                               f"(layout {tuned['rb']['chosen']})",
                     "launches": launches,
                     "kernel_ms_per_launch": ms_per_launch,
                     "alg_bytes_per_launch": bytes_per_launch},
    }
    if args.learned_train > 0:
        # time-to-all-solutions, learned vs first-fail (untimed leg, same GPU,
        # same layout and launch for both policies)
        from paper_1909_09213_amd import learn
        rep = learn.experiment(ctx, n_train=args.learned_train, n_eval=args.learned_eval)
        rep.pop("theta")
        out["learned_vs_first_fail"] = rep
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
