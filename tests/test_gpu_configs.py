"""GPU parity at the benchmark configurations' shapes.

* global family (all-different + linear <=): exact counts on scaled twins;
  at full size (200 vars over 0..255, 65,536 initial subproblems, count cap
  10^6) the capped count and the verifier on every returned solution;
* batched find-first sweep (instances of uneven size in one persistent
  launch): verdicts against the oracle wherever the oracle resolves the
  instance within its node budget, and every SAT assignment verified;
* the random binary configuration: 13-queens and RB slices against the
  oracle, and slice sums against a full GPU count.
"""
import sys

import numpy as np
import pytest

import cspgen
import oracle

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


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------ global family

@pytest.mark.parametrize("idx", range(3))
def test_global_twin_exact(ctx, cb, idx):
    inst = cspgen.global_twin(idx)
    _say("global twin", idx)
    ref = oracle.solve(inst, oracle.MODE_COUNT)
    for split in (0, 4096):
        r = ctx.solve(ctx.load(inst), cb.MODE_COUNT, split_target=split)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), split


def test_global_twin_all_solutions(ctx, cb):
    inst = cspgen.global_twin(1, n=7, d=8, k_ad=4)
    ref = oracle.solve(inst, oracle.MODE_ALL, sol_cap=200000)
    r = ctx.solve(ctx.load(inst), cb.MODE_ALL, sol_capacity=ref.count)
    assert r.count == ref.count
    got = sorted(map(tuple, r.solutions.tolist()))
    want = sorted(map(tuple, ref.solutions.tolist()))
    assert got == want


def test_global_full_size_capped(ctx, cb):
    inst = cspgen.global_family(0)
    assert inst.n == 200 and int(inst.dsize.max()) == 256
    _say("global full size, cap 1e6, split 65536")
    r = ctx.solve(ctx.load(inst), cb.MODE_COUNT, max_solutions=10 ** 6, split_target=65536,
                  sol_capacity=1000)
    assert r.verdict == "LIMIT" and r.count == 10 ** 6
    assert r.n_written == 1000
    rows = {tuple(x) for x in r.solutions.tolist()}
    assert len(rows) == 1000  # pairwise distinct
    for row in r.solutions:
        assert oracle.verify(inst, row)
    # the oracle agrees the instance is satisfiable (capped)
    ref = oracle.solve(inst, oracle.MODE_COUNT, cap=5)
    assert ref.count == 5


# -------------------------------------------------------------- batch sweep

def _sweep(B, base=cspgen.SEED_SWEEP, **ranges):
    return [cspgen.rb_sweep(i, base=base, **ranges) for i in range(B)]


@pytest.mark.parametrize("layout", [1, 2])
def test_batch_first_small_vs_oracle(ctx, cb, layout):
    insts = _sweep(48, nhi=40, dhi=24)
    probs = [ctx.load(x) for x in insts]
    res = ctx.solve_batch(probs, cb.MODE_FIRST, layout=layout)
    resolved = 0
    for inst, r in zip(insts, res):
        ref = oracle.solve(inst, oracle.MODE_FIRST, max_nodes=200000)
        if ref.verdict != "LIMIT":
            resolved += 1
            assert r.verdict == ref.verdict, inst.name
        if r.verdict == "SAT":
            assert oracle.verify(inst, r.solutions[0]), inst.name
        else:
            assert r.verdict == "UNSAT"
    assert resolved >= 24


def test_batch_count_matches_single(ctx, cb):
    insts = _sweep(16, nlo=12, nhi=20, dlo=5, dhi=9, plo=350, phi=550, tlo=300, thi=450, base=99)
    probs = [ctx.load(x) for x in insts]
    res = ctx.solve_batch(probs, cb.MODE_COUNT, max_nodes=50_000_000)
    resolved = 0
    for inst, r in zip(insts, res):
        ref = oracle.solve(inst, oracle.MODE_COUNT, max_nodes=300000)
        if ref.verdict != "LIMIT":
            resolved += 1
            assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), inst.name
    assert resolved >= 8


def test_batch_full_size(ctx, cb):
    """4096 instances, n in [20,120], d in [8,64], in one persistent launch."""
    insts = _sweep(4096)
    _say("generated 4096 sweep instances")
    probs = [ctx.load(x) for x in insts]
    _say("loaded")
    res = ctx.solve_batch(probs, cb.MODE_FIRST, max_nodes=200_000, layout=1)
    n_sat = n_unsat = 0
    for inst, r in zip(insts, res):
        if r.verdict == "SAT":
            n_sat += 1
            assert oracle.verify(inst, r.solutions[0]), inst.name
        elif r.verdict == "UNSAT":
            n_unsat += 1
    _say(f"batch: sat={n_sat} unsat={n_unsat} kernel_ms={res[0].kernel_ms:.1f}")
    assert n_sat + n_unsat > 2048
    # seeded sample checked against the oracle (budgeted)
    rng = np.random.default_rng(3)
    agree = 0
    for i in rng.choice(4096, 24, replace=False):
        ref = oracle.solve(insts[i], oracle.MODE_FIRST, max_nodes=20000)
        if ref.verdict != "LIMIT" and res[i].verdict != "LIMIT":
            assert ref.verdict == res[i].verdict, insts[i].name
            agree += 1
    assert agree >= 8


# ---------------------------------------------------- random binary config

def test_queens13_count_and_nodes(ctx, cb):
    inst = cspgen.queens(13)
    ref = oracle.solve(inst, oracle.MODE_COUNT)
    r = ctx.solve(ctx.load(inst), cb.MODE_COUNT)
    assert r.count == 73712 == ref.count
    assert (r.nodes, r.fails) == (ref.nodes, ref.fails)


def test_rb_full_size_sampled_subproblems(ctx, cb):
    """RB n=40, d=16: exact parity on seeded sub-CSPs the oracle finishes."""
    inst = cspgen.rb(0)
    rng = np.random.default_rng(11)
    for _ in range(6):
        vals = rng.integers(0, 16, 5)
        sub = inst.fix({i: int(v) for i, v in enumerate(vals)})
        ref = oracle.solve(sub, oracle.MODE_COUNT)
        r = ctx.solve(ctx.load(sub), cb.MODE_COUNT)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails)


def test_rb_slices_sum_to_full_count(ctx, cb):
    """Slices x0 = v partition the search tree (GPU only, any size)."""
    inst = cspgen.rb(4, n=28, d=10, dens_pm=250, tight_pm=380)
    failed, bits, _ = oracle.root(inst)
    assert not failed and all(int(b[0]) == (1 << 10) - 1 for b in bits)
    full = ctx.solve(ctx.load(inst), cb.MODE_COUNT)
    parts = [ctx.solve(ctx.load(inst.fix({0: v})), cb.MODE_COUNT) for v in range(10)]
    assert sum(p.count for p in parts) == full.count
    assert sum(p.nodes for p in parts) == full.nodes - 1
