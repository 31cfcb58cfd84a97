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
import os
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


BENCH_BUDGET = 50_000  # node budget per instance of the benchmark's batch


def _sweep_golden():
    rows = _golden_rows("sweep_verdicts.txt")
    assert len(rows) == 4096
    out = {}
    for r in rows:
        out[int(r[0])] = (r[1], int(r[2]), int(r[3]))
    return out


def _check_batch_against_oracle(insts, res, sols, golden, tag):
    """Every GPU SAT assignment verified; every instance both sides resolve
    with the same verdict; every oracle UNSAT (a whole first-fail tree of at
    most 20,000 nodes, within the GPU's budget) UNSAT on the GPU with the
    same node and failure counts.  An instance the oracle finds satisfiable
    may still end at the GPU's budget: many workers share its tree and
    explore other subtrees than the oracle's leftmost path before one of
    them reaches a solution.  Returns (GPU UNSAT verdicts the oracle left
    unresolved, oracle-SAT instances the GPU left at its budget)."""
    n_sat = n_unsat = unchecked = sat_at_budget = 0
    for b, (inst, r) in enumerate(zip(insts, res)):
        v, nodes, fails = golden[b]
        if r.verdict == "SAT":
            n_sat += 1
            assert oracle.verify(inst, sols[b, :inst.n]), (tag, inst.name)
        elif r.verdict == "UNSAT":
            n_unsat += 1
            unchecked += v == "LIMIT"
        if v != "LIMIT" and r.verdict != "LIMIT":
            assert r.verdict == v, (tag, inst.name, r.verdict, v)
        if v == "SAT" and r.verdict == "LIMIT":
            sat_at_budget += 1
        if v == "UNSAT":
            assert r.verdict == "UNSAT", (tag, inst.name, r.verdict)
            assert (r.nodes, r.fails) == (nodes, fails), (tag, inst.name)
    _say(f"{tag}: sat={n_sat} unsat={n_unsat} (oracle-unresolved unsat {unchecked}) "
         f"limit={len(res) - n_sat - n_unsat} (oracle-sat {sat_at_budget}) kernel_ms={res[0].kernel_ms:.0f}")
    return unchecked, sat_at_budget


def test_batch_full_size(ctx, cb):
    """The benchmark's batch: 4096 instances (n in [20,120], d in [8,64])
    in one persistent launch, find-first, a node budget of 50,000 each,
    with the autotuned layout, then once more replayed from a hipGraph.
    Checked on every instance against the oracle's stored verdicts (budget
    20,000 nodes each, tests/golden/sweep_verdicts.txt)."""
    import torch
    golden = _sweep_golden()
    insts = _sweep(4096)
    _say("generated 4096 sweep instances")
    probs = [ctx.load(x) for x in insts]
    _say("loaded")
    nmax = max(x.n for x in insts)
    sol = torch.zeros((4096, nmax), dtype=torch.int32, device=ctx.torch_device)
    chosen = ctx.autotune(probs, cb.MODE_FIRST, time_ms=300, max_nodes=BENCH_BUDGET)
    _say(f"autotuned layout {chosen}")
    for tag, kw in (("autotuned", {}), ("graph", {"use_graph": True}), ("graph replay", {"use_graph": True})):
        sol.zero_()
        res = ctx.solve_batch(probs, cb.MODE_FIRST, max_nodes=BENCH_BUDGET, sol_out=sol, **kw)
        s = sol.cpu().numpy()
        unchecked, sat_at_budget = _check_batch_against_oracle(insts, res, s, golden, tag)
        assert unchecked <= 64, unchecked
        assert sat_at_budget <= 41, sat_at_budget  # at most 1% of the instances
    resolved = sum(v != "LIMIT" for v, _, _ in golden.values())
    _say(f"oracle resolved {resolved} of 4096 within 20,000 nodes")
    assert resolved >= 2500


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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_rows(name):
    """Data rows of a stored oracle result (tests/golden/make_goldens.py)."""
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def test_rb_bench_slice_partition(ctx, cb):
    """The benchmark's RB slice x0 = 1 (n=40, d=16, tightness 0.35): its
    full GPU count equals the oracle's count summed over the 16 sub-CSPs
    x1 = v, and every sub-CSP's count, node and failure counts equal the
    oracle's (stored, tests/golden/rb_slice_x0_1.txt)."""
    inst = cspgen.rb(0, n=40, d=16, dens_pm=250, tight_pm=350, base=cspgen.SEED_RB)
    rows = {int(r[0]): tuple(int(x) for x in r[1:]) for r in _golden_rows("rb_slice_x0_1.txt")}
    assert sorted(rows) == list(range(16))
    full = ctx.solve(ctx.load(inst.fix({0: 1})), cb.MODE_COUNT)
    _say(f"RB slice x0=1: {full.count} solutions, {full.nodes} nodes, {full.kernel_ms:.0f} ms")
    assert full.verdict == "SAT" and full.count == sum(r[0] for r in rows.values())
    for v in range(16):
        r = ctx.solve(ctx.load(inst.fix({0: 1, 1: v})), cb.MODE_COUNT)
        assert (r.count, r.nodes, r.fails) == rows[v], v


def test_rb_bench_depth2_subproblems(ctx, cb):
    """Seeded sub-CSPs of the benchmark's RB instance with x0 and x1 fixed
    (about 10^9 nodes each): count, node and failure counts equal the
    oracle's (stored, tests/golden/rb_depth2.txt)."""
    inst = cspgen.rb(0, n=40, d=16, dens_pm=250, tight_pm=350, base=cspgen.SEED_RB)
    rows = _golden_rows("rb_depth2.txt")
    assert len(rows) >= 6
    for a, b, count, nodes, fails in ([int(x) for x in r] for r in rows):
        r = ctx.solve(ctx.load(inst.fix({0: a, 1: b})), cb.MODE_COUNT)
        assert (r.count, r.nodes, r.fails) == (count, nodes, fails), (a, b)


def test_rb_tightness_040_full_count(ctx, cb):
    """RB n=40, d=16 at tightness 0.40 (102 of 256 pairs forbidden per
    table) counted exhaustively: count, nodes and failures equal the
    oracle's (stored, tests/golden/rb_tight400.txt)."""
    inst = cspgen.rb(0, n=40, d=16, dens_pm=250, tight_pm=400, base=cspgen.SEED_RB)
    want = {r[0]: int(r[1]) for r in _golden_rows("rb_tight400.txt")}
    for layout in (0, 1, 3):
        r = ctx.solve(ctx.load(inst), cb.MODE_COUNT, layout=layout)
        assert (r.count, r.nodes, r.fails) == (want["count"], want["nodes"], want["fails"]), layout


def test_rb_slices_sum_to_full_count(ctx, cb):
    """Slices x0 = v partition the search tree (GPU only, any size)."""
    inst = cspgen.rb(4, n=28, d=10, dens_pm=250, tight_pm=380)
    failed, bits, _ = oracle.root(inst)
    assert not failed and all(int(b[0]) == (1 << 10) - 1 for b in bits)
    full = ctx.solve(ctx.load(inst), cb.MODE_COUNT)
    parts = [ctx.solve(ctx.load(inst.fix({0: v})), cb.MODE_COUNT) for v in range(10)]
    assert sum(p.count for p in parts) == full.count
    assert sum(p.nodes for p in parts) == full.nodes - 1
