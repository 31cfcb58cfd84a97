"""Learned variable ordering: trace collection, GPU training, evaluation.

1. collect(): solve instances with the plain first-fail solver in count
   mode, one instance per worker (no donation, no split, so every subtree is
   searched by one worker and its size is exact), with a fraction of the
   branchings exploring among the 4 smallest domains.  Every completed
   subtree below a branching yields a record (5 features of the branching
   variable, depth, label = log2(1 + nodes below)).
2. train(): full-batch Adam on the GPU with the library's own forward /
   backward / optimizer kernels (bf16 MFMA forward, fp32 master weights).
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
        out.append(buf[:n].clone())
        total += n
        for p in probs:
            p.free()
        if total >= cap:
            break
    return torch.cat(out, 0) if out else torch.zeros((0, 8), device=ctx.torch_device)


def train(ctx: cb.Context, rec, steps: int = 300, lr: float = 3e-3, seed: int = 0,
          theta=None, log_every: int = 0):
    """Train the policy on trace records with full-batch Adam on the GPU."""
    pol = cb.Policy(ctx, init_theta(seed) if theta is None else theta)
    losses = []
    for s in range(1, steps + 1):
        loss = pol.train_step(rec, lr, s)
        losses.append(loss)
        if log_every and s % log_every == 0:
            print(f"step {s} loss {loss:.4f}", flush=True)
    return pol, losses


def evaluate(ctx: cb.Context, insts, policy, mode: int = cb.MODE_COUNT, max_nodes: int = 0):
    """Solve every instance under first-fail and under the policy (one batched
    launch each).  Returns per-policy totals and per-instance results."""
    probs = [ctx.load(x) for x in insts]
    out = {}
    for name, br, pol in (("first_fail", cb.BRANCH_FIRST_FAIL, None),
                          ("learned", cb.BRANCH_LEARNED, policy)):
        t0 = time.perf_counter()
        res = ctx.solve_batch(probs, mode, branching=br, policy=pol, max_nodes=max_nodes)
        dt = time.perf_counter() - t0
        out[name] = {"results": res, "nodes": sum(r.nodes for r in res),
                     "kernel_ms": res[0].kernel_ms, "wall_s": dt}
    for p in probs:
        p.free()
    return out
