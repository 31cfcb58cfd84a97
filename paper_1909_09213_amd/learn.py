"""Learned variable ordering: search traces, GPU training, evaluation.

1. Traces of the plain solver.  Two kinds, both produced by the library:
   - collect(): count-mode solves, one instance per worker (no donation, no
     split, so every subtree is searched by one worker and its size is
     exact), a fraction of the branchings exploring among the 4 smallest
     domains; every completed subtree below a branching yields a record (5
     features of the branching variable, depth, instance, label =
     log2(1 + nodes below)).  These are observational: each node has one
     branching, and a regression on them learns what instance and depth do
     to subtree sizes (first-fail branches on high-degree variables near
     the root, where subtrees are large, so degree comes out as predicting
     LARGER subtrees - the opposite of what shrinks the tree).
   - sample_nodes() + sibling_records(): at sampled search nodes, the
     subtree below branching on EACH of several candidate variables is
     counted by the plain solver (every child x = v solved exhaustively in
     one batched launch).  Records of one node differ only in the choice of
     variable; this is what the policy is trained on.
2. train(): labels centred per group of column 6 / column 5 (node id and
   depth for sibling records; instance and depth for collect()'s), so the
   network learns how the choice of variable moves the subtree size at a
   node; every candidate at a node shares the group, so the argmin is
   unchanged by the centring.  Then full-batch Adam on the GPU with the
   library's own forward / backward / optimizer kernels (bf16 MFMA forward,
   fp32 master weights).
3. evaluate(): the same held-out instances under first-fail and under the
   learned policy; verdicts and counts must agree, nodes and time compared.

Only the solver library is used here; nothing calls the CPU oracle.
"""
from __future__ import annotations

import time

import numpy as np

import cspgen

from . import cubics as cb

NP = 449
F, H = 5, 64


def init_theta(seed: int = 0) -> np.ndarray:
    """He-style initial parameters: W1[64][5], b1, w2, b2."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NP, dtype=np.float32)
    th[0:H * F] = rng.normal(0, np.sqrt(2.0 / F), H * F)
    th[H * F:H * F + H] = 0.01
    th[H * F + H:H * F + 2 * H] = rng.normal(0, np.sqrt(1.0 / H), H)
    return th


# The learned-branching workload: tractable-count instances of the batched
# sweep generator (n, d, density, tightness drawn per instance from reduced
# ranges so that every instance's complete search tree fits a trace run).
LEARN_RANGES = dict(nlo=16, nhi=28, dlo=6, dhi=12, plo=350, phi=550, tlo=300, thi=450)


def instances(base: int, count: int, **ranges):
    r = dict(LEARN_RANGES)
    r.update(ranges)
    return [cspgen.rb_sweep(i, base=base, **r) for i in range(count)]


def global_instances(base: int, count: int):
    """The learned-branching workload of the all-different + linear family,
    at sizes whose trees can be counted exhaustively: per instance n in
    {8, 9} variables over 0..d-1 with d in {6, 7, 8} (drawn from the
    instance seed), two all-different constraints over ceil(n/2) variables
    each and three linear <= constraints over all variables, b = 45% of the
    largest sum (the full family's rules)."""
    out = []
    for i in range(count):
        r = int(cspgen.rng_below(cspgen.instance_seed(base, i), 6, 1)[0])
        n, d = 8 + r // 3, 6 + r % 3
        out.append(cspgen.global_family(i, n=n, lo=0, d=d, n_ad=2, k_ad=(n + 1) // 2, n_lin=3, lin_k=0,
                                        amax=9, b_pm=450, base=base))
    return out


FAMILIES = {"sweep": instances, "global": global_instances}


def collect(ctx: cb.Context, insts, cap: int = 4_000_000, explore_pm: int = 250, seed: int = 1,
            chunk: int = 2048, max_nodes: int = 2_000_000):
    """Trace records [N, 8] (torch float32 on the device)."""
    import torch
    out = []
    total = 0
    for c0 in range(0, len(insts), chunk):
        part = insts[c0:c0 + chunk]
        probs = [ctx.load(x) for x in part]
        buf = torch.zeros((cap - total, 8), dtype=torch.float32, device=ctx.torch_device)
        res = ctx.solve_batch(probs, cb.MODE_COUNT, donate=False, max_nodes=max_nodes,
                              trace=buf, explore_pm=explore_pm, seed=seed + c0)
        n = min(res[0].traces, buf.shape[0])
        part_rec = buf[:n].clone()
        part_rec[:, 6] += c0  # instance index within the whole list
        out.append(part_rec)
        total += n
        for p in probs:
            p.free()
        if total >= cap:
            break
    return torch.cat(out, 0) if out else torch.zeros((0, 8), device=ctx.torch_device)


def sample_nodes(ctx: cb.Context, insts, seed: int = 0):
    """One search node per instance: a random descent from the root (the
    branching variable by first-fail on half of the steps, else uniform among
    the unassigned; the value uniform), propagated on the GPU after every
    branching, to a depth drawn uniformly in [1, n/2]; a branching whose
    propagation fails is redrawn (up to 4 times), then the descent stops at
    its last consistent node.  Returns (index, depth, domains) with the
    fixpoint domains of the node ([n, W] words)."""
    rng = np.random.default_rng(seed)
    out = []
    for k, inst in enumerate(insts):
        target = int(rng.integers(1, max(2, inst.n // 2 + 1)))
        prob = ctx.load(inst)
        failed, dom = ctx.root(prob, device_words=True)
        prob.free()
        if failed:
            continue
        depth = 0
        while depth < target:
            pops = np.array([sum(bin(int(w)).count("1") for w in row) for row in dom])
            free = np.flatnonzero(pops >= 2)
            if free.size == 0:
                break
            child = None
            for _ in range(4):
                if rng.integers(0, 2) == 0:
                    x = int(free[np.lexsort((free, pops[free]))[0]])
                else:
                    x = int(rng.choice(free))
                vals = [32 * w + b for w in range(dom.shape[1]) for b in range(32)
                        if (int(dom[x, w]) >> b) & 1]
                a = int(rng.choice(vals))
                init = dom.copy()
                init[x] = 0
                init[x, a // 32] = np.uint32(1 << (a % 32))
                prob = ctx.load(inst.with_init(init[:, :inst.W]))
                failed, c = ctx.root(prob, device_words=True)
                prob.free()
                if not failed:
                    child = c
                    break
            if child is None:
                break
            dom, depth = child, depth + 1
        if depth >= 1:
            out.append((k, depth, dom))
    return out


def sibling_records(ctx: cb.Context, insts, nodes, n_small: int = 6, n_other: int = 2,
                    max_nodes: int = 2_000_000, seed: int = 0, chunk: int = 4096):
    """Subtree sizes of alternative branchings at the same node, from the
    plain solver: at each sampled node, for each candidate variable x (the
    n_small smallest domains and n_other others, uniformly), every child
    x = v is counted exhaustively in one batched launch; the subtree below
    branching on x holds sum_v nodes(child v).  Records [N, 8] (torch,
    device): features of x at the node, depth, node id, label
    log2(1 + subtree size).  Nodes with a child over max_nodes are dropped."""
    import torch
    rng = np.random.default_rng(seed)
    jobs = []  # (node id, x, child init)
    feats = {}
    for nid, (k, depth, dom) in enumerate(nodes):
        inst = insts[k]
        pops = np.array([sum(bin(int(w)).count("1") for w in row) for row in dom])
        free = np.flatnonzero(pops >= 2)
        if free.size < 2:
            continue
        order = free[np.lexsort((free, pops[free]))]
        cands = list(order[:n_small])
        rest = order[n_small:]
        if rest.size:
            cands += list(rng.choice(rest, size=min(n_other, rest.size), replace=False))
        prob = ctx.load(inst.with_init(dom[:, :inst.W]))
        feats[nid] = (ctx.features(prob, dom, depth), depth)
        prob.free()
        for x in cands:
            x = int(x)
            for w in range(dom.shape[1]):
                for b in range(32):
                    if (int(dom[x, w]) >> b) & 1:
                        init = dom[:, :inst.W].copy()
                        init[x] = 0
                        init[x, w] = np.uint32(1 << b)
                        jobs.append((nid, x, inst, init))
    size = {}
    over = set()
    for c0 in range(0, len(jobs), chunk):
        part = jobs[c0:c0 + chunk]
        probs = [ctx.load(inst.with_init(init)) for _, _, inst, init in part]
        res = ctx.solve_batch(probs, cb.MODE_COUNT, max_nodes=max_nodes)
        for (nid, x, _, _), r in zip(part, res):
            if r.verdict == "LIMIT":
                over.add(nid)
            size[(nid, x)] = size.get((nid, x), 0) + r.nodes
        for p in probs:
            p.free()
    rows = []
    for (nid, x), sz in size.items():
        if nid in over:
            continue
        f, depth = feats[nid]
        rows.append(list(f[x]) + [float(depth), float(nid), float(np.log2(1.0 + sz))])
    rec = np.asarray(rows, dtype=np.float32).reshape(-1, 8)
    return torch.from_numpy(rec).to(ctx.torch_device)


def value_records(ctx: cb.Context, insts, nodes, max_nodes: int = 2_000_000, chunk: int = 4096):
    """Training records of the value network, from the plain solver: at each
    sampled node, the first-fail variable x and, for every value a of x, the
    number of solutions below the child x = a (counted exhaustively, all
    children in batched launches).  Records [N, 8] (torch, device): the
    value's 5 features at the node (cubics_value_features), depth, node id,
    label log2(1 + solutions below x = a).  Nodes with a child over
    max_nodes, or with domains wider than 64 values, are dropped."""
    import torch
    jobs = []  # (node id, value, instance, child init)
    feats = {}
    for nid, (k, depth, dom) in enumerate(nodes):
        inst = insts[k]
        if dom.shape[1] > 2:
            continue
        pops = np.array([sum(bin(int(w)).count("1") for w in row) for row in dom])
        free = np.flatnonzero(pops >= 2)
        if free.size == 0:
            continue
        x = int(free[np.lexsort((free, pops[free]))[0]])
        prob = ctx.load(inst.with_init(dom[:, :inst.W]))
        feats[nid] = (ctx.value_features(prob, dom, depth, x), depth)
        prob.free()
        for w in range(dom.shape[1]):
            for bit in range(32):
                if (int(dom[x, w]) >> bit) & 1:
                    init = dom[:, :inst.W].copy()
                    init[x] = 0
                    init[x, w] = np.uint32(1 << bit)
                    jobs.append((nid, 32 * w + bit, inst, init))
    sols = {}
    over = set()
    for c0 in range(0, len(jobs), chunk):
        part = jobs[c0:c0 + chunk]
        probs = [ctx.load(inst.with_init(init)) for _, _, inst, init in part]
        res = ctx.solve_batch(probs, cb.MODE_COUNT, max_nodes=max_nodes)
        for (nid, a, _, _), r in zip(part, res):
            if r.verdict == "LIMIT":
                over.add(nid)
            sols[(nid, a)] = r.count
        for p in probs:
            p.free()
    rows = []
    for (nid, a), cnt in sols.items():
        if nid in over:
            continue
        f, depth = feats[nid]
        rows.append(list(f[a]) + [float(depth), float(nid), float(np.log2(1.0 + cnt))])
    rec = np.asarray(rows, dtype=np.float32).reshape(-1, 8)
    return torch.from_numpy(rec).to(ctx.torch_device)


def evaluate_first(ctx: cb.Context, insts, vpolicy, max_nodes: int = 2_000_000):
    """Find-first under the ascending value order and under the value
    network, each instance searched by one worker (no donation: the same
    depth-first order every run), all instances in one launch per order.
    Returns per-order results and launch times; raises if a verdict differs
    between the two orders where both resolve the instance."""
    probs = [ctx.load(x) for x in insts]
    out = {}
    for name, vp in (("ascending", None), ("learned", vpolicy)):
        res = ctx.solve_batch(probs, cb.MODE_FIRST, donate=False, max_nodes=max_nodes,
                              layout=cb.LAYOUT_LANE, value_policy=vp)
        out[name] = {"results": res, "kernel_ms": res[0].kernel_ms}
    for i, (a, b) in enumerate(zip(out["ascending"]["results"], out["learned"]["results"])):
        if a.verdict != "LIMIT" and b.verdict != "LIMIT" and a.verdict != b.verdict:
            raise AssertionError(f"value order changed the verdict of instance {i}")
    for p in probs:
        p.free()
    return out


def value_experiment(ctx: cb.Context, n_train: int = 2000, n_eval: int = 1024, steps: int = 1500,
                     lr: float = 1e-2, train_base: int = cspgen.SEED_TRAIN + 2000,
                     eval_base: int = cspgen.SEED_EVAL + 2000, family: str = "sweep"):
    """Train the value network on solution counts below the children of the
    first-fail variable at one sampled node of each of n_train instances,
    then find a first solution of n_eval held-out instances under the
    ascending order and under the network.  Report: nodes to the first
    solution on the instances both orders solve (satisfiable ones whose
    ascending search takes at least n + 1 nodes, i.e. backtracks), their
    geometric-mean ratio, and the launch times."""
    make = FAMILIES[family]
    t0 = time.perf_counter()
    train_insts = make(train_base, n_train)
    nodes = sample_nodes(ctx, train_insts, seed=train_base)
    rec = value_records(ctx, train_insts, nodes)
    t_label = time.perf_counter() - t0
    del train_insts
    t0 = time.perf_counter()
    vpol, losses = train(ctx, rec, steps=steps, lr=lr)
    t_train = time.perf_counter() - t0
    held = make(eval_base, n_eval)
    ev = evaluate_first(ctx, held, vpol)
    asc, lrn = ev["ascending"]["results"], ev["learned"]["results"]
    sat = [i for i in range(n_eval) if asc[i].verdict == "SAT" and lrn[i].verdict == "SAT"]
    hard = [i for i in sat if asc[i].nodes > held[i].n + 1]
    r_all = np.array([lrn[i].nodes / asc[i].nodes for i in sat], dtype=np.float64)
    r_hard = np.array([lrn[i].nodes / asc[i].nodes for i in hard], dtype=np.float64)
    c7 = centre_labels(rec)[:, 7].double()
    return {
        "family": family, "train_instances": n_train, "records": int(rec.shape[0]),
        "label_variance": float((c7 * c7).mean().item()) if c7.numel() else None,
        "loss_first": losses[0], "loss_last": losses[-1],
        "eval_instances": n_eval, "sat_both": len(sat), "backtracking_sat": len(hard),
        "unsat_both": sum(asc[i].verdict == "UNSAT" and lrn[i].verdict == "UNSAT" for i in range(n_eval)),
        "nodes_to_first_ascending": int(sum(asc[i].nodes for i in sat)),
        "nodes_to_first_learned": int(sum(lrn[i].nodes for i in sat)),
        "node_ratio_geomean_sat": float(np.exp(np.mean(np.log(r_all)))) if len(sat) else None,
        "node_ratio_geomean_backtracking": float(np.exp(np.mean(np.log(r_hard)))) if len(hard) else None,
        "fewer_nodes": int((r_hard < 1).sum()), "more_nodes": int((r_hard > 1).sum()),
        "launch_ms_ascending": ev["ascending"]["kernel_ms"], "launch_ms_learned": ev["learned"]["kernel_ms"],
        "seconds": {"label": t_label, "train": t_train},
        "theta": vpol.get().tolist(),
    }


def centre_labels(rec):
    """Copy of the records with column 7 replaced by the label minus the mean
    label of its (instance, depth) group."""
    import torch
    key = rec[:, 6].to(torch.int64) * 65536 + rec[:, 5].to(torch.int64)
    _, inv = torch.unique(key, return_inverse=True)
    g = int(inv.max().item()) + 1 if inv.numel() else 0
    s = torch.zeros(g, dtype=torch.float64, device=rec.device).index_add_(0, inv, rec[:, 7].double())
    c = torch.zeros(g, dtype=torch.float64, device=rec.device).index_add_(
        0, inv, torch.ones_like(rec[:, 7], dtype=torch.float64))
    out = rec.clone()
    out[:, 7] = (rec[:, 7].double() - (s / c)[inv]).float()
    return out


def train(ctx: cb.Context, rec, steps: int = 300, lr: float = 3e-3, seed: int = 0,
          theta=None, log_every: int = 0, centre: bool = True):
    """Train the policy on trace records with full-batch Adam on the GPU."""
    if centre:
        rec = centre_labels(rec)
    if theta is None:
        theta = init_theta(seed)
        # a feature that is constant in the data gets no gradient: start it
        # (and keep it) at zero weight instead of a random one
        const = (rec[:, :F].max(0).values - rec[:, :F].min(0).values).cpu().numpy() == 0
        W1 = theta[:H * F].reshape(H, F)
        W1[:, const] = 0.0
    pol = cb.Policy(ctx, theta)
    losses = []
    for s in range(1, steps + 1):
        loss = pol.train_step(rec, lr, s)
        losses.append(loss)
        if log_every and s % log_every == 0:
            print(f"step {s} loss {loss:.4f}", flush=True)
    return pol, losses


def evaluate(ctx: cb.Context, insts, policy, mode: int = cb.MODE_COUNT, max_nodes: int = 0,
             repeats: int = 3):
    """Solve every instance under first-fail and under the policy (one batched
    launch each, both in the LANE layout, which the learned path uses).
    Returns per-policy totals and per-instance results.  With a node budget,
    the instances first-fail resolves within it are solved again (budget x8)
    in one launch per policy: "resolved_kernel_ms" is the
    time-to-all-solutions of that set (the budget-capped launches are
    dominated by instances that stop at the budget, where both policies do
    the same number of nodes); the fastest of `repeats` launches, since a
    launch's time is that of its largest trees and varies between runs."""
    probs = [ctx.load(x) for x in insts]
    out = {}
    for name, br, pol in (("first_fail", cb.BRANCH_FIRST_FAIL, None),
                          ("learned", cb.BRANCH_LEARNED, policy)):
        t0 = time.perf_counter()
        res = ctx.solve_batch(probs, mode, branching=br, policy=pol, max_nodes=max_nodes,
                              layout=cb.LAYOUT_LANE)
        dt = time.perf_counter() - t0
        out[name] = {"results": res, "nodes": sum(r.nodes for r in res),
                     "kernel_ms": res[0].kernel_ms, "wall_s": dt}
    if max_nodes:
        keep = [i for i, r in enumerate(out["first_fail"]["results"]) if r.verdict != "LIMIT"]
        sub = [probs[i] for i in keep]
        out["resolved_by_first_fail"] = keep
        # the launch's time is that of its tail (its largest trees), which
        # varies between identical launches: the fastest of `repeats`
        for name, br, pol in (("first_fail", cb.BRANCH_FIRST_FAIL, None),
                              ("learned", cb.BRANCH_LEARNED, policy)):
            times = []
            res = []
            for _ in range(repeats if sub else 0):
                res = ctx.solve_batch(sub, mode, branching=br, policy=pol, layout=cb.LAYOUT_LANE,
                                      max_nodes=8 * max_nodes)
                times.append(res[0].kernel_ms)
            out[name]["resolved_kernel_ms"] = min(times) if times else 0.0
            out[name]["resolved_kernel_ms_all"] = times
            out[name]["resolved_nodes"] = sum(r.nodes for r in res)
            out[name]["resolved_over_8x_budget"] = sum(r.verdict == "LIMIT" for r in res)
        # time-to-all of single instances: the first `single` resolved ones,
        # each in its own launch under both policies
        single = keep[:128]
        ratios = []
        for i in single:
            t = []
            for br, pol in ((cb.BRANCH_FIRST_FAIL, None), (cb.BRANCH_LEARNED, policy)):
                r = ctx.solve(probs[i], mode, branching=br, policy=pol, layout=cb.LAYOUT_LANE,
                              max_nodes=8 * max_nodes)
                t.append(r.kernel_ms)
            ratios.append(t[1] / max(t[0], 1e-6))
        out["single_instances"] = len(single)
        out["single_time_ratio_geomean"] = float(np.exp(np.mean(np.log(ratios)))) if ratios else None
    for p in probs:
        p.free()
    return out


def experiment(ctx: cb.Context, n_train: int = 20000, n_eval: int = 4096, steps: int = 1500,
               lr: float = 1e-2, eval_max_nodes: int = 50_000_000,
               train_base: int = cspgen.SEED_TRAIN, eval_base: int = cspgen.SEED_EVAL,
               family: str = "sweep"):
    """Sample one node from each of n_train seeded instances of `family`
    ("sweep": the batched random binary generator at reduced sizes;
    "global": the all-different + linear generator at reduced sizes), label
    the alternative branchings there with the plain solver's subtree sizes,
    train, and evaluate time-to-all (count mode) on n_eval held-out seeds
    under first-fail and the policy.  Returns a report dict; raises if any
    verdict or count differs."""
    make = FAMILIES[family]
    t0 = time.perf_counter()
    train_insts = make(train_base, n_train)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    nodes = sample_nodes(ctx, train_insts, seed=train_base)
    rec = sibling_records(ctx, train_insts, nodes, seed=train_base)
    t_collect = time.perf_counter() - t0
    del train_insts
    t0 = time.perf_counter()
    pol, losses = train(ctx, rec, steps=steps, lr=lr)
    t_train = time.perf_counter() - t0
    eval_insts = make(eval_base, n_eval)
    ev = evaluate(ctx, eval_insts, pol, cb.MODE_COUNT, max_nodes=eval_max_nodes)
    ff, le = ev["first_fail"]["results"], ev["learned"]["results"]
    both = [i for i in range(n_eval) if ff[i].verdict != "LIMIT" and le[i].verdict != "LIMIT"]
    for i in both:
        if ff[i].count != le[i].count or ff[i].verdict != le[i].verdict:
            raise AssertionError(f"policy changed the count of eval instance {i}")
    nodes_ff = sum(ff[i].nodes for i in both)
    nodes_le = sum(le[i].nodes for i in both)
    ratios = np.array([le[i].nodes / ff[i].nodes for i in both], dtype=np.float64)
    c7 = centre_labels(rec)[:, 7].double()
    report = {
        "family": family,
        "train_instances": n_train, "train_nodes": len(nodes), "eval_instances": n_eval,
        "label_variance": float((c7 * c7).mean().item()) if c7.numel() else None,
        "eval_resolved_by_both": len(both),
        "records": int(rec.shape[0]), "train_steps": steps,
        "loss_first": losses[0], "loss_last": losses[-1],
        "nodes_first_fail": nodes_ff, "nodes_learned": nodes_le,
        "node_ratio_learned_over_ff": nodes_le / max(nodes_ff, 1),
        "node_ratio_geomean": float(np.exp(np.mean(np.log(ratios)))) if len(both) else None,
        "instances_fewer_nodes": int((ratios < 1).sum()),
        "instances_more_nodes": int((ratios > 1).sum()),
        "budget_per_instance": eval_max_nodes,
        "capped_launch_ms_first_fail": ev["first_fail"]["kernel_ms"],
        "capped_launch_ms_learned": ev["learned"]["kernel_ms"],
        "resolved_by_first_fail": len(ev["resolved_by_first_fail"]),
        "time_to_all_ms_first_fail": ev["first_fail"]["resolved_kernel_ms"],
        "time_to_all_ms_learned": ev["learned"]["resolved_kernel_ms"],
        "time_to_all_ms_runs_first_fail": ev["first_fail"]["resolved_kernel_ms_all"],
        "time_to_all_ms_runs_learned": ev["learned"]["resolved_kernel_ms_all"],
        "time_ratio_learned_over_ff": ev["learned"]["resolved_kernel_ms"]
        / max(ev["first_fail"]["resolved_kernel_ms"], 1e-9),
        "resolved_nodes_first_fail": ev["first_fail"]["resolved_nodes"],
        "resolved_nodes_learned": ev["learned"]["resolved_nodes"],
        "resolved_over_8x_budget_learned": ev["learned"]["resolved_over_8x_budget"],
        "single_instance_launches": ev["single_instances"],
        "single_instance_time_ratio_geomean": ev["single_time_ratio_geomean"],
        "seconds": {"generate": t_gen, "label": t_collect, "train": t_train},
        "theta": pol.get().tolist(),
    }
    return report


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--eval", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=1500)
    args = ap.parse_args()
    ctx = cb.Context(0)
    rep = experiment(ctx, n_train=args.train, n_eval=args.eval, steps=args.steps)
    theta = rep.pop("theta")
    print(json.dumps(rep))
