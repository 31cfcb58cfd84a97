"""Learned branching on the GPU: forward, gradients and Adam of the policy
network's kernels against the fp64 reference; the policy changes node counts
but never verdicts, counts or solution sets."""
import sys

import numpy as np
import pytest

import cspgen
import oracle
from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    from paper_1909_09213_amd import cubics
    return cubics


@pytest.fixture(scope="module")
def ctx(cb):
    c = cb.Context(0)
    yield c
    c.close()


def _rec(N, seed):
    rng = np.random.default_rng(seed)
    rec = np.zeros((N, 8), dtype=np.float32)
    rec[:, 0] = rng.uniform(0, 1, N)
    rec[:, 1] = rng.uniform(0, 0.5, N)
    rec[:, 2] = rng.uniform(0, 0.6, N)
    rec[:, 3] = rng.uniform(0, 1, N)
    rec[:, 4] = np.log2(1 + rng.integers(0, 50, N))
    rec[:, 7] = rng.uniform(0, 12, N)
    return rec


def test_forward_matches_reference(ctx, cb):
    import torch
    th = M.init_theta(3)
    pol = cb.Policy(ctx, th)
    rec = _rec(1000, 1)
    y = pol.forward(torch.from_numpy(rec).to(ctx.torch_device)).cpu().numpy()
    ref, _, _ = M.forward(th, rec[:, :5], quantized=True)
    assert np.allclose(y, ref, rtol=2e-2, atol=1e-3), np.max(np.abs(y - ref))


def test_gradient_matches_reference(ctx, cb):
    import torch
    th = M.init_theta(5)
    pol = cb.Policy(ctx, th)
    rec = _rec(3000, 2)
    g, loss = pol.grad(torch.from_numpy(rec).to(ctx.torch_device))
    g = g.cpu().numpy()
    ref = M.grad(th, rec[:, :5], rec[:, 7], quantized=True)
    scale = np.max(np.abs(ref))
    assert np.all(np.abs(g - ref) <= 2e-2 * np.abs(ref) + 1e-3 * scale), np.max(np.abs(g - ref) / scale)
    lref = M.loss(th, rec[:, :5], rec[:, 7], quantized=True)
    assert abs(float(loss.item()) - lref) <= 2e-2 * lref


def test_adam_step_matches_reference(ctx, cb):
    import torch
    th0 = M.init_theta(7)
    pol = cb.Policy(ctx, th0)
    rec = _rec(2000, 3)
    X = torch.from_numpy(rec).to(ctx.torch_device)
    lr = 1e-2
    pol.train_step(X, lr, 1)
    got = pol.get().astype(np.float64)
    g = M.grad(th0, rec[:, :5], rec[:, 7], quantized=True)
    want, _, _ = M.adam_step(th0.astype(np.float64), np.zeros(M.NP), np.zeros(M.NP), g, lr, 1)
    # a first Adam step moves every parameter by lr * g / (|g| + eps): compare
    # where the gradient is clearly non-zero, bound the move elsewhere
    big = np.abs(g) > 1e-2 * np.max(np.abs(g))
    assert np.allclose(got[big], want[big], rtol=0, atol=1e-4)
    assert np.all(np.abs(got - th0) <= lr * (1 + 1e-3))


def test_learned_policy_keeps_counts_and_verdicts(ctx, cb):
    th = M.init_theta(11)
    pol = cb.Policy(ctx, th)
    insts = [cspgen.rb_sweep(i, base=123, nlo=12, nhi=18, dlo=5, dhi=9, plo=350, phi=550,
                             tlo=300, thi=450) for i in range(32)]
    probs = [ctx.load(x) for x in insts]
    ff = ctx.solve_batch(probs, cb.MODE_COUNT)
    lr = ctx.solve_batch(probs, cb.MODE_COUNT, branching=cb.BRANCH_LEARNED, policy=pol)
    differ = 0
    for inst, a, b in zip(insts, ff, lr):
        assert a.verdict != "LIMIT" and b.verdict != "LIMIT"
        assert a.count == b.count, inst.name
        ref = oracle.solve(inst, oracle.MODE_COUNT, max_nodes=300000)
        if ref.verdict != "LIMIT":
            assert a.count == ref.count, inst.name
        differ += a.nodes != b.nodes
    assert differ > 0  # the policy does change the search order
    fa = ctx.solve_batch(probs, cb.MODE_FIRST)
    fb = ctx.solve_batch(probs, cb.MODE_FIRST, branching=cb.BRANCH_LEARNED, policy=pol)
    for inst, a, b in zip(insts, fa, fb):
        assert a.verdict == b.verdict
        if b.verdict == "SAT":
            assert oracle.verify(inst, b.solutions[0])
    # all-solutions sets under the policy equal the oracle's
    q = cspgen.queens(7)
    r = ctx.solve(ctx.load(q), cb.MODE_ALL, sol_capacity=64, branching=cb.BRANCH_LEARNED, policy=pol)
    ref = oracle.solve(q, oracle.MODE_ALL, sol_cap=64)
    assert sorted(map(tuple, r.solutions.tolist())) == sorted(map(tuple, ref.solutions.tolist()))


def _first_fail_policy():
    """A closed-form network: one live hidden unit reading feature 0
    (|D_i| / d_i) with weight 1, output weight 1, every other parameter 0.
    Its prediction is the domain fraction itself (bf16-exact when d is 8 or
    16, and strictly increasing in |D_i| for any one d), so on instances
    whose variables share one domain size its argmin (lowest index on ties)
    is the first-fail choice."""
    th = np.zeros(M.NP, dtype=np.float32)
    th[M.OFF_W1 + 0 * M.F + 0] = 1.0
    th[M.OFF_W2 + 0] = 1.0
    return th


@pytest.mark.parametrize("inst_fn", [lambda: cspgen.queens(8), lambda: cspgen.queens(10),
                                     lambda: cspgen.rb(5, n=16, d=16, dens_pm=350, tight_pm=560),
                                     lambda: cspgen.rb(6, n=18, d=8, dens_pm=350, tight_pm=410)],
                         ids=["queens8", "queens10", "rb_d16", "rb_d8"])
def test_closed_form_policy_is_first_fail(ctx, cb, inst_fn):
    """The fused in-kernel network and argmin pick exactly the first-fail
    variable: node and failure counts equal the oracle's first-fail search,
    with one worker and with the device full of workers."""
    inst = inst_fn()
    assert len(set(int(x) for x in inst.dsize)) == 1
    pol = cb.Policy(ctx, _first_fail_policy())
    ref = oracle.solve(inst, oracle.MODE_COUNT)
    prob = ctx.load(inst)
    for kw in ({"workers": 1}, {}):
        r = ctx.solve(prob, cb.MODE_COUNT, branching=cb.BRANCH_LEARNED, policy=pol, **kw)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), kw


def test_trace_collection_and_training(ctx, cb):
    from paper_1909_09213_amd import learn
    insts = learn.instances(base=cspgen.SEED_TRAIN, count=256)
    rec = learn.collect(ctx, insts, cap=500000, explore_pm=250)
    print(f"traces: {rec.shape[0]}", file=sys.stderr, flush=True)
    assert rec.shape[0] > 1000
    r = rec.cpu().numpy()
    assert np.all(r[:, 7] >= 0) and np.all(np.isfinite(r))
    assert np.all((r[:, 0] > 0) & (r[:, 0] <= 1))
    assert np.all((r[:, 6] == np.floor(r[:, 6])) & (r[:, 6] >= 0) & (r[:, 6] < len(insts)))
    # labels centred per (instance, depth): zero mean in every group
    c = learn.centre_labels(rec).cpu().numpy()
    key = r[:, 6].astype(np.int64) * 65536 + r[:, 5].astype(np.int64)
    sums = np.bincount(np.unique(key, return_inverse=True)[1], weights=c[:, 7])
    assert np.max(np.abs(sums)) < 1e-2 * max(1.0, float(np.abs(c[:, 7]).sum()) / len(sums))
    pol, losses = learn.train(ctx, rec, steps=150, lr=1e-2)
    # the network explains part of the centred labels' variance (the loss of
    # the best constant predictor, 0)
    var0 = float(np.mean(c[:, 7].astype(np.float64) ** 2))
    print(f"loss {losses[0]:.3f} -> {losses[-1]:.3f}, constant predictor {var0:.3f}", file=sys.stderr)
    assert losses[-1] < losses[0] and losses[-1] < 0.98 * var0


def test_features_match_their_definition(ctx, cb):
    """cubics_features against the features written out from the instance:
    |D_i| / d_i, (number of constraints on i) / (n - 1), mean over i's
    tables of the forbidden fraction, depth / n, log2(1 + 0)."""
    inst = cspgen.rb_sweep(7, base=321, nlo=14, nhi=18, dlo=5, dhi=9, plo=300, phi=500,
                           tlo=300, thi=450)
    n = inst.n
    deg = np.zeros(n)
    tsum = np.zeros(n)
    for c in range(inst.m):
        i, j = (int(v) for v in inst.scope(c))
        di, dj = int(inst.dsize[i]), int(inst.dsize[j])
        bits = np.unpackbits(inst.tab(c).view(np.uint8), bitorder="little").reshape(di, -1)[:, :dj]
        t = 1.0 - bits.sum() / (di * dj)
        for v in (i, j):
            deg[v] += 1
            tsum[v] += t
    sub = inst.fix({0: int(inst.lo[0]), 3: int(inst.lo[3]) + 1})
    p = ctx.load(sub)
    failed, dom = ctx.root(p, device_words=True)
    assert not failed
    got = ctx.features(p, dom, depth=2)
    pop = np.array([sum(bin(int(w)).count("1") for w in row) for row in dom])
    want = np.stack([pop / inst.dsize, deg / (n - 1), np.where(deg > 0, tsum / np.maximum(deg, 1), 0),
                     np.full(n, 2 / n), np.zeros(n)], axis=1)
    assert np.allclose(got, want, rtol=1e-6, atol=1e-7), np.max(np.abs(got - want))
    # NULL domains = the initial ones
    got0 = ctx.features(p, None, depth=0)
    pop0 = np.array([sum(bin(int(w)).count("1") for w in row) for row in sub.init])
    assert pop0[0] == 1 and pop0[3] == 1 and pop0[1] == inst.dsize[1]
    assert np.allclose(got0[:, 0], pop0 / inst.dsize, rtol=1e-6)
    assert np.all(got0[:, 3] == 0)


def test_trained_policy_gains_over_first_fail(ctx, cb):
    """Train on sibling subtree sizes at nodes of 600 seeded instances, then
    count 256 held-out instances under first-fail and under the policy (same
    layout, same launch): identical counts, and fewer nodes on most
    instances (the geometric mean of the per-instance node ratios)."""
    from paper_1909_09213_amd import learn
    train = learn.instances(cspgen.SEED_TRAIN, 600)
    nodes = learn.sample_nodes(ctx, train, seed=1)
    rec = learn.sibling_records(ctx, train, nodes, seed=1)
    pol, losses = learn.train(ctx, rec, steps=800, lr=1e-2)
    # the network explains a real part of the centred labels' variance (the
    # loss of the best constant predictor)
    c = learn.centre_labels(rec)[:, 7].double()
    var0 = float((c * c).mean().item())
    assert losses[-1] < 0.8 * var0, (losses[-1], var0)
    held = learn.instances(cspgen.SEED_EVAL, 256)
    ev = learn.evaluate(ctx, held, pol, cb.MODE_COUNT, max_nodes=20_000_000)
    ff, le = ev["first_fail"]["results"], ev["learned"]["results"]
    both = [i for i in range(len(held)) if ff[i].verdict != "LIMIT" and le[i].verdict != "LIMIT"]
    assert len(both) >= 200
    for i in both:
        assert (ff[i].count, ff[i].verdict) == (le[i].count, le[i].verdict), held[i].name
    r = np.array([le[i].nodes / ff[i].nodes for i in both])
    geo = float(np.exp(np.mean(np.log(r))))
    print(f"records {rec.shape[0]}, loss {losses[0]:.3f} -> {losses[-1]:.3f}; node ratio geomean "
          f"{geo:.3f}, fewer {int((r < 1).sum())}, more {int((r > 1).sum())}; kernel ms "
          f"{ev['first_fail']['kernel_ms']:.0f} -> {ev['learned']['kernel_ms']:.0f}", file=sys.stderr)
    assert geo < 0.9
    assert (r < 1).sum() > 2 * (r > 1).sum()


def test_global_family_policy_keeps_counts(ctx, cb):
    """The all-different + linear family at countable sizes: a policy
    trained on sibling subtree sizes of 300 instances counts 128 held-out
    instances exactly as first-fail does (same counts and verdicts; node
    counts may differ)."""
    from paper_1909_09213_amd import learn
    train = learn.global_instances(cspgen.SEED_TRAIN + 1000, 300)
    nodes = learn.sample_nodes(ctx, train, seed=2)
    rec = learn.sibling_records(ctx, train, nodes, seed=2)
    assert rec.shape[0] > 500
    pol, losses = learn.train(ctx, rec, steps=400, lr=1e-2)
    assert losses[-1] < losses[0]
    held = learn.global_instances(cspgen.SEED_EVAL + 1000, 128)
    ev = learn.evaluate(ctx, held, pol, cb.MODE_COUNT, max_nodes=20_000_000)
    ff, le = ev["first_fail"]["results"], ev["learned"]["results"]
    both = [i for i in range(len(held)) if ff[i].verdict != "LIMIT" and le[i].verdict != "LIMIT"]
    assert len(both) == len(held)
    for i in both:
        assert (ff[i].count, ff[i].verdict) == (le[i].count, le[i].verdict), held[i].name
    for i in range(0, len(held), 16):
        ref = oracle.solve(held[i], oracle.MODE_COUNT)
        assert ff[i].count == ref.count, held[i].name
    r = np.array([le[i].nodes / ff[i].nodes for i in both])
    print(f"global family: node ratio geomean {float(np.exp(np.mean(np.log(r)))):.3f}", file=sys.stderr)
