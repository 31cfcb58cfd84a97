"""Measurements of every configuration on one GPU, one JSON object per line.

    python -m paper_1909_09213_amd.report [--learned-train N] [--learned-eval M]

  8-queens        all solutions (92), nodes, kernel time
  queens13        count (73,712), nodes, kernel time
  rb_slice        one x0-slice of the n=40 d=16 RB instance, nodes/s per layout
  batch_sweep     4096 sweep instances, find-first, one launch, autotuned
                  layout and worker count, per-instance node budget
  global_capped   n=200 d=256 all-different + linear, count capped at 10^6,
                  split into 65,536 subproblems
  learned         traces -> GPU training -> learned vs first-fail node counts
                  and time-to-all on held-out seeds (same layout, same launch)
  lns             large-neighbourhood search minimising the sum of the
                  variables of an RB instance (n=60, d=12): objective per round

Every count and verdict the library returns is checked where a closed value
is known (queens); parity against the oracle is the tests' business.
"""
from __future__ import annotations

import argparse
import json
import time

import cspgen

from . import cubics as cb
from . import learn


def _emit(obj):
    print(json.dumps(obj), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--learned-train", type=int, default=2000)
    ap.add_argument("--learned-eval", type=int, default=512)
    ap.add_argument("--learned-steps", type=int, default=1500)
    ap.add_argument("--skip", default="", help="comma-separated names to skip")
    args = ap.parse_args()
    skip = set(filter(None, args.skip.split(",")))
    ctx = cb.Context(0)

    for n, want in ((8, 92), (13, 73712)):
        name = "8-queens" if n == 8 else "queens13"
        if name in skip:
            continue
        p = ctx.load(cspgen.queens(n))
        lay, div, rates = ctx.autotune([p], cb.MODE_COUNT, time_ms=100, rates=True)
        mode = cb.MODE_ALL if n == 8 else cb.MODE_COUNT
        r = ctx.solve(p, mode, sol_capacity=want if n == 8 else 0)
        assert r.count == want, (name, r.count)
        _emit({"config": name, "count": r.count, "nodes": r.nodes, "fails": r.fails,
               "kernel_ms": r.kernel_ms, "wall_ms": r.ms, "layout": lay, "worker_divisor": div})

    if "rb_slice" not in skip:
        p = ctx.load(cspgen.rb(0).fix({0: 15}))
        out = {"config": "rb_slice", "slice": "x0=15", "time_ms": 2000}
        for lay, name in ((1, "lane"), (2, "seg"), (3, "var")):
            r = ctx.solve(p, cb.MODE_COUNT, layout=lay, time_ms=2000)
            out[name + "_nodes_per_s"] = r.nodes / (r.kernel_ms * 1e-3)
            out[name + "_revisions_per_node"] = r.revisions / max(r.nodes, 1)
        _emit(out)

    if "batch_sweep" not in skip:
        insts = [cspgen.rb_sweep(i) for i in range(4096)]
        probs = [ctx.load(x) for x in insts]
        budget = 200_000
        lay, div, rates = ctx.autotune(probs, cb.MODE_FIRST, time_ms=300, rates=True, max_nodes=budget)
        t0 = time.perf_counter()
        res = ctx.solve_batch(probs, cb.MODE_FIRST, max_nodes=budget)
        wall = time.perf_counter() - t0
        v = [r.verdict for r in res]
        nodes = sum(r.nodes for r in res)
        _emit({"config": "batch_sweep", "instances": 4096, "node_budget": budget,
               "sat": v.count("SAT"), "unsat": v.count("UNSAT"), "limit": v.count("LIMIT"),
               "nodes": nodes, "kernel_ms": res[0].kernel_ms, "wall_s": wall,
               "nodes_per_s": nodes / (res[0].kernel_ms * 1e-3),
               "layout": lay, "worker_divisor": div,
               "autotune_nodes_per_ms": {f"{k[0]}/{k[1]}": round(x) for k, x in rates.items()}})
        for p in probs:
            p.free()

    if "global_capped" not in skip:
        p = ctx.load(cspgen.global_family(0))
        r = ctx.solve(p, cb.MODE_COUNT, max_solutions=10 ** 6, split_target=65536)
        _emit({"config": "global_capped", "count": r.count, "verdict": r.verdict, "nodes": r.nodes,
               "fails": r.fails, "tasks": r.tasks, "kernel_ms": r.kernel_ms,
               "nodes_per_s": r.nodes / (r.kernel_ms * 1e-3)})

    if "lns" not in skip:
        inst = cspgen.rb(5, n=60, d=12, dens_pm=200, tight_pm=300)
        obj = [1] * inst.n
        trace = []
        for rounds in (1, 2, 4, 8, 16):
            r = ctx.lns(inst, obj, neighborhoods=1024, relax_pm=200, max_nodes=20000, rounds=rounds, seed=7)
            trace.append({"rounds": r["rounds"], "objective": r["objective"], "ms": round(r["ms"], 1),
                          "nodes": r["nodes"], "optimal": r["optimal"]})
        _emit({"config": "lns", "instance": "RB n=60 d=12 density 0.2 tightness 0.3, minimise sum x",
               "neighborhoods": 1024, "relax_pm": 200, "max_nodes_per_copy": 20000, "runs": trace})

    if "learned" not in skip:
        rep = learn.experiment(ctx, n_train=args.learned_train, n_eval=args.learned_eval,
                               steps=args.learned_steps)
        rep.pop("theta")
        rep["config"] = "learned"
        _emit(rep)


if __name__ == "__main__":
    main()
