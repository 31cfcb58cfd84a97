"""Benchmark: search nodes/s and constraint revisions/s on one MI355X.

Headline workload (the batched plain-solving configuration): 4096 seeded
random binary CSPs of uneven size - per instance n ~ U{20..120} variables,
d ~ U{8..64} values (one or two 32-bit words per domain), density ~ U{0.1..0.3}
and tightness ~ U{0.2..0.5} (base seed 3, indices 0..4095) - solved in
find-first mode, all 4096 in one persistent launch, with a node budget per
instance (--budget, default 50,000: an instance still unresolved after that
many nodes stops with verdict LIMIT; the tightness sweep crosses the
satisfiability transition, where instances can take exponentially many
nodes).  The revision layout and worker count are the library's autotuned
choice for the batch.  One step = one launch over the whole batch; the
instances are loaded on the device before the timed region.

The JSON line reports nodes/s (value) and revisions/s over the timed steps,
the roofline of the search kernel (algorithmic domain / table-row / trail
bytes per launch, counted by the kernel, over the launch's duration measured
with HIP events on the library's stream; HBM traffic from the committed
rocprofv3 counter summary when it was taken on the current kernel source),
and the CPU oracle timed on the same instances (one core, and one process per
core of the host's CPU share).  Further legs, each reported with its own
figures and outside the timed region: 8-queens all solutions, the RB n=40
d=16 count configuration (one top-level slice) and 13-queens, the
all-different + linear family (count capped at 10^6, 65,536 initial
subproblems), the learned-vs-first-fail branching experiment on both
generators, and the learned value order against ascending values
(find-first).
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
BATCH = 4096
KERNEL_SOURCES = ["paper_1909_09213_amd/csrc/cubics_search.hip",
                  "paper_1909_09213_amd/csrc/cubics_internal.h",
                  "paper_1909_09213_amd/csrc/cubics_host.cpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_kernel_sweep_traffic.json")
METRIC = "search nodes/s + revisions/s at 1 GPU; time-to-all-solutions learned vs first-fail"


def say(msg: str) -> None:
    """Progress line on stderr (the JSON line is the only stdout output)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch(budget: int):
    """HBM bytes per batch launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and budget."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("budget") != budget:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Cores of this process's CPU share (at most 16: a one-GPU machine's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _oracle_part(args):
    """One CPU process: the oracle on batch instances `idxs` (find-first,
    per-instance node budget) until `deadline` (time.time()); returns
    (nodes, revisions, instances, seconds inside the oracle)."""
    idxs, budget, deadline = args
    import cspgen
    import oracle
    nodes = revs = k = 0
    t_used = 0.0
    for i in idxs:
        if time.time() >= deadline:
            break
        inst = cspgen.rb_sweep(int(i))
        t0 = time.perf_counter()
        r = oracle.solve(inst, oracle.MODE_FIRST, max_nodes=budget)
        t_used += time.perf_counter() - t0
        nodes += r.nodes
        revs += r.revisions
        k += 1
    return nodes, revs, k, t_used


def cpu_baseline(budget_s: float, node_budget: int):
    """The oracle (plain single-threaded AC-3 + chronological backtracking)
    on the headline batch's instances, in a seeded order, each with a node
    budget of node_budget: one process for ~budget_s seconds, then one
    process per core for ~budget_s seconds of wall time.  Runs before the
    GPU is initialised (the pool forks)."""
    import multiprocessing as mp

    import numpy as np
    order = np.random.default_rng(20240).permutation(BATCH)
    nodes, revs, k, t_used = _oracle_part((order, node_budget, time.time() + budget_s))
    one = {"value": nodes / t_used, "unit": "nodes/s", "cores": 1, "kind": "oracle",
           "revisions_per_s": revs / t_used,
           "sample": f"oracle find-first on {k} batch instances (seeded order, node budget "
                     f"{node_budget} each): {nodes} nodes in {t_used:.1f} s"}
    cores = host_cores()
    parts = [(order[c::cores], node_budget, 0.0) for c in range(cores)]
    t0 = time.time()
    deadline = t0 + budget_s
    parts = [(p[0], p[1], deadline) for p in parts]
    with mp.get_context("fork").Pool(cores) as pool:
        outs = pool.map(_oracle_part, parts)
    wall = time.time() - t0
    an = sum(o[0] for o in outs)
    ar = sum(o[1] for o in outs)
    ak = sum(o[2] for o in outs)
    one["all_cores"] = {"value": an / wall, "unit": "nodes/s", "cores": cores,
                        "revisions_per_s": ar / wall,
                        "sample": f"{cores} oracle processes over a static split of the same "
                                  f"order: {ak} instances, {an} nodes in {wall:.1f} s wall"}
    one["cpu_model"] = cpu_model()
    return one


def leg_queens8(ctx, cb, cspgen):
    p = ctx.load(cspgen.queens(8))
    r = ctx.solve(p, cb.MODE_ALL, sol_capacity=128)
    assert r.count == 92, r.count
    return {"workload": "8-queens, all solutions", "count": r.count, "nodes": r.nodes,
            "fails": r.fails, "kernel_ms": round(r.kernel_ms, 3)}


def leg_rb(ctx, cb, cspgen):
    """RB n=40 d=16 (195 tables, 90/256 pairs forbidden, seed 2 index 0):
    the top-level slice x0 = 1 counted exhaustively, then 13-queens."""
    inst = cspgen.rb(0, n=40, d=16, dens_pm=250, tight_pm=350, base=cspgen.SEED_RB)
    tune = ctx.load(inst.fix({0: 15}))
    chosen, div, rates = ctx.autotune([tune], cb.MODE_COUNT, time_ms=400, rates=True)
    names = {1: "lane", 2: "seg", 3: "var"}
    sl = ctx.load(inst.fix({0: 1}))
    r = ctx.solve(sl, cb.MODE_COUNT)
    q13 = ctx.load(cspgen.queens(13))
    qchosen, qdiv = ctx.autotune([q13], cb.MODE_COUNT, time_ms=100, rates=True)[:2]
    q = ctx.solve(q13, cb.MODE_COUNT)
    assert q.count == 73712, q.count
    return {"workload": "model-RB n=40 d=16 density 0.25 tightness 0.35 (seed 2 index 0), "
                        "slice x0=1 count-all; 13-queens count-all",
            "layout": names[chosen], "worker_divisor": div,
            "slice_count": r.count, "slice_nodes": r.nodes, "slice_kernel_ms": round(r.kernel_ms, 3),
            "slice_nodes_per_s": r.nodes / (r.kernel_ms * 1e-3),
            "slice_revisions_per_s": r.revisions / (r.kernel_ms * 1e-3),
            "slice_alg_GBps": r.alg_bytes / (r.kernel_ms * 1e-3) / 1e9,
            "queens13_count": q.count, "queens13_nodes": q.nodes,
            "queens13_layout": names[qchosen], "queens13_worker_divisor": qdiv,
            "queens13_kernel_ms": round(q.kernel_ms, 3)}


def leg_global(ctx, cb, cspgen):
    inst = cspgen.global_family(0)
    r = ctx.solve(ctx.load(inst), cb.MODE_COUNT, max_solutions=10 ** 6, split_target=65536)
    assert r.count == 10 ** 6, r.count
    return {"workload": "200 vars over 0..255, 10 all-different x 20 vars, 30 linear <= "
                        "(seed 4 index 0), count capped at 10^6, 65,536 initial subproblems",
            "count": r.count, "verdict": r.verdict, "nodes": r.nodes, "tasks": r.tasks,
            "fails": r.fails, "kernel_ms": round(r.kernel_ms, 3),
            "nodes_per_s": r.nodes / (r.kernel_ms * 1e-3)}


def leg_linear_ad(ctx, cb, cspgen):
    """Linear <= bounded with the all-different groups in its scope against
    the plain bound: 256 global twins (8 vars over 0..7, 2 all-different x 5,
    3 linear <=) counted exhaustively in one batch, and the full global
    instance's count capped at 10^6."""
    twins = [cspgen.global_twin(i) for i in range(256)]
    out = {"workload": "256 global twins (n=8, d=8, 2 all-different x 5, 3 linear <=) count-all; "
                       "global family (seed 4 index 0) count capped at 10^6"}
    counts = {}
    for tag, insts in (("plain", twins), ("linear_ad", [x.with_linear_ad() for x in twins])):
        probs = [ctx.load(x) for x in insts]
        res = ctx.solve_batch(probs, cb.MODE_COUNT)
        counts[tag] = [r.count for r in res]
        out[f"twins_{tag}_nodes"] = sum(r.nodes for r in res)
        out[f"twins_{tag}_fails"] = sum(r.fails for r in res)
        out[f"twins_{tag}_kernel_ms"] = round(res[0].kernel_ms, 3)
        for p in probs:
            p.free()
    assert counts["plain"] == counts["linear_ad"]
    g = ctx.load(cspgen.global_family(0).with_linear_ad())
    r = ctx.solve(g, cb.MODE_COUNT, max_solutions=10 ** 6, split_target=65536)
    assert r.count == 10 ** 6, r.count
    out.update({"global_linear_ad_nodes": r.nodes, "global_linear_ad_fails": r.fails,
                "global_linear_ad_kernel_ms": round(r.kernel_ms, 3)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget", type=int, default=50_000, help="node budget per instance")
    ap.add_argument("--layout", type=int, default=0, help="0 autotuned, 1 lane, 2 seg")
    ap.add_argument("--cpu-budget", type=float, default=10.0,
                    help="seconds of each CPU-oracle run (one core, then all cores)")
    ap.add_argument("--cpu-node-budget", type=int, default=2000,
                    help="node budget per instance of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 8-queens, RB, global-family and learned legs")
    ap.add_argument("--learned-train", type=int, default=2000,
                    help="training instances of the learned-vs-first-fail leg (0 = skip it)")
    ap.add_argument("--learned-eval", type=int, default=512)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 256 MiB device-to-device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; --gpus must be 1 (sharding a "
              "search over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.budget < 1:
        print("bench.py: need steps >= 1, warmup >= 0, budget >= 1", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu:
        say("CPU oracle baseline")
        cpu = cpu_baseline(args.cpu_budget, args.cpu_node_budget)
        say(f"CPU oracle: {cpu['value']:.0f} nodes/s on 1 core, "
            f"{cpu['all_cores']['value']:.0f} on {cpu['all_cores']['cores']}")

    import torch

    import cspgen
    from paper_1909_09213_amd import cubics as cb

    t_setup = time.perf_counter()
    ctx = cb.Context(0)
    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    say("generating and loading the batch")
    insts = [cspgen.rb_sweep(i) for i in range(BATCH)]
    probs = [ctx.load(x) for x in insts]
    nmax = max(x.n for x in insts)
    del insts
    sol_out = torch.zeros((BATCH, nmax), dtype=torch.int32, device="cuda")
    names = {1: "lane", 2: "seg", 3: "var"}
    tuned = None
    if args.layout == 0:
        # the library's autotuner: every admitted layout x worker count on the
        # batch itself, in 400 ms windows (untimed)
        say("autotuning the batch")
        chosen, div, rates = ctx.autotune(probs, cb.MODE_FIRST, time_ms=400, rates=True,
                                          max_nodes=args.budget)
        tuned = {"chosen": names[chosen], "worker_divisor": div,
                 "active_per_xcd": ctx.last_active_per_xcd,
                 "nodes_per_ms": {f"{names[k]}/{d}": round(v) for (k, d), v in rates.items()}}
    t_setup = time.perf_counter() - t_setup

    def step(tag):
        res = ctx.solve_batch(probs, cb.MODE_FIRST, max_nodes=args.budget, layout=args.layout,
                              sol_out=sol_out)
        say(f"{tag}: {res[0].kernel_ms:.0f} ms")
        return res

    for w in range(args.warmup):
        step(f"warmup {w + 1}/{args.warmup}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(f"step {s + 1}/{args.steps}") for s in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    nodes = sum(r.nodes for res in runs for r in res)
    revs = sum(r.revisions for res in runs for r in res)
    bytes_per_launch = sum(r.alg_bytes for res in runs for r in res) / len(runs)
    kms = [res[0].kernel_ms for res in runs]
    ms_per_launch = sum(kms) / len(kms)
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    traffic = traffic_per_launch(args.budget)
    last = runs[-1]
    verdicts = {v: sum(r.verdict == v for r in last) for v in ("SAT", "UNSAT", "LIMIT")}
    out = {
        "metric": METRIC,
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
        "config": {"workload": f"{BATCH} random binary CSPs (n U[20,120], d U[8,64], density "
                               f"U[0.1,0.3], tightness U[0.2,0.5], seed 3 indices 0..{BATCH - 1}), "
                               f"find-first, one persistent launch per step, node budget "
                               f"{args.budget} per instance",
                   "batch": BATCH, "budget": args.budget, "layout": args.layout,
                   "autotuned": tuned},
        "revisions_per_s": revs / dt,
        "verdicts_last_step": verdicts,
        "nodes_per_step": [sum(r.nodes for r in res) for res in runs],
        "kernel_ms": [round(x, 3) for x in kms],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "search_kernel, one launch over the 4096-instance batch",
                     "launches": len(runs), "kernel_ms_per_launch": ms_per_launch,
                     "alg_bytes_per_launch": bytes_per_launch,
                     "traffic_GBps": (traffic / (ms_per_launch * 1e-3) / 1e9) if traffic else None},
        "setup_s": round(t_setup, 2),
    }
    for p in probs:
        p.free()
    del probs
    if not args.no_extras:
        legs = {}
        for name, fn in (("queens8", leg_queens8), ("rb_count", leg_rb), ("global", leg_global),
                         ("linear_ad", leg_linear_ad)):
            say(f"leg {name}")
            t = time.perf_counter()
            legs[name] = fn(ctx, cb, cspgen)
            legs[name]["seconds"] = round(time.perf_counter() - t, 2)
        out["legs"] = legs
        if args.learned_train > 0:
            # time-to-all-solutions, learned vs first-fail (same GPU, same
            # layout and launch for both policies)
            from paper_1909_09213_amd import learn
            out["learned_vs_first_fail"] = {}
            for fam in ("sweep", "global"):
                say(f"leg learned_vs_first_fail ({fam})")
                t = time.perf_counter()
                rep = learn.experiment(ctx, n_train=args.learned_train, n_eval=args.learned_eval,
                                       family=fam)
                rep.pop("theta")
                rep["seconds_total"] = round(time.perf_counter() - t, 2)
                out["learned_vs_first_fail"][fam] = rep
            # the learned value order (find-first): nodes to the first
            # solution against ascending values, one worker per instance
            say("leg learned_value_order (sweep)")
            t = time.perf_counter()
            rep = learn.value_experiment(ctx, n_train=4 * args.learned_train, n_eval=2 * args.learned_eval)
            rep.pop("theta")
            rep["seconds_total"] = round(time.perf_counter() - t, 2)
            out["learned_value_order"] = rep
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
