"""GPU parity: the HIP solver against the CPU oracle on the same seeded
instances.  Bit-exact everywhere: root fixpoint domains, solution sets and
counts, node and failure counts in all/count mode; in first mode the verdict
plus an assignment the independent verifier accepts."""
import sys

import numpy as np
import pytest

import cspgen
import oracle

pytestmark = pytest.mark.gpu

LAYOUTS = [1, 2, 3]  # LANE, SEG, VAR


@pytest.fixture(scope="module")
def cb():
    from paper_1909_09213_amd import cubics
    return cubics


@pytest.fixture(scope="module")
def ctx(cb):
    c = cb.Context(0)
    yield c
    c.close()


def _canon(rows):
    return sorted(tuple(int(v) for v in r) for r in rows)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check_all(ctx, cb, inst, layout, workers=0, split=0):
    ref = oracle.solve(inst, oracle.MODE_ALL, sol_cap=20000)
    prob = ctx.load(inst)
    r = ctx.solve(prob, cb.MODE_ALL, layout=layout, sol_capacity=max(ref.count, 1),
                  workers=workers, split_target=split)
    assert r.count == ref.count, (inst.name, r.count, ref.count)
    assert (r.nodes, r.fails) == (ref.nodes, ref.fails), (inst.name, r.nodes, ref.nodes, r.fails, ref.fails)
    assert r.verdict == ref.verdict
    if ref.count <= 20000:
        assert _canon(r.solutions) == _canon(ref.solutions), inst.name
    return r


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("form", [0, 1])
def test_worked_example(ctx, cb, layout, form):
    inst = cspgen.worked_example(form)
    _say("worked example", form, layout)
    failed, bits = ctx.root(ctx.load(inst), layout)
    rf, rbits, _ = oracle.root(inst)
    assert failed == rf and np.array_equal(bits, rbits)
    r = _check_all(ctx, cb, inst, layout)
    assert r.count == 11 and r.nodes == 14 and r.fails == 0
    f = ctx.solve(ctx.load(inst), cb.MODE_FIRST, layout=layout)
    assert f.verdict == "SAT" and oracle.verify(inst, f.solutions[0])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_nqueens_all(ctx, cb, layout):
    for n in range(1, 11):
        _say("queens", n, layout)
        _check_all(ctx, cb, cspgen.queens(n), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_8queens_single_worker_and_split(ctx, cb, layout):
    inst = cspgen.queens(8)
    _check_all(ctx, cb, inst, layout, workers=1)
    _check_all(ctx, cb, inst, layout, workers=7)
    _check_all(ctx, cb, inst, layout, split=40)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_random_mixed(ctx, cb, layout):
    for idx in range(60):
        inst = cspgen.mixed(idx + 9000, n=6, dmax=7, m=8)
        _say("mixed", idx, layout)
        failed, bits = ctx.root(ctx.load(inst), layout)
        rf, rbits, _ = oracle.root(inst)
        assert failed == rf, idx
        if not rf:
            assert np.array_equal(bits, rbits), idx
        _check_all(ctx, cb, inst, layout)
        f = ctx.solve(ctx.load(inst), cb.MODE_FIRST, layout=layout)
        ref = oracle.solve(inst, oracle.MODE_COUNT)
        assert f.verdict == ("SAT" if ref.count else "UNSAT")
        if f.verdict == "SAT":
            assert oracle.verify(inst, f.solutions[0])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_root_fixpoint_rb_and_sweep(ctx, cb, layout):
    insts = [cspgen.rb(0), cspgen.rb(1, tight_pm=450), cspgen.rb(2, n=30, d=12, tight_pm=500)]
    insts += [cspgen.rb_sweep(i) for i in range(6)]
    for inst in insts:
        _say("root", inst.name, layout)
        failed, bits = ctx.root(ctx.load(inst), layout)
        rf, rbits, _ = oracle.root(inst)
        assert failed == rf
        if not rf:
            assert np.array_equal(bits, rbits), inst.name


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rb_small_count(ctx, cb, layout):
    for idx in range(4):
        inst = cspgen.rb(idx, n=20, d=8, dens_pm=300, tight_pm=390)
        _say("rb small", idx, layout)
        ref = oracle.solve(inst, oracle.MODE_COUNT)
        r = ctx.solve(ctx.load(inst), cb.MODE_COUNT, layout=layout)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails)


def test_edge_cases(ctx, cb):
    empty = cspgen.Instance(lo=np.zeros(0, np.int32), dsize=np.zeros(0, np.int32),
                            type=np.zeros(0, np.int32), arity=np.zeros(0, np.int32),
                            var_off=np.zeros(1, np.int64), vars=np.zeros(0, np.int32),
                            par_off=np.zeros(1, np.int64), params=np.zeros(0, np.int64),
                            tab_off=np.zeros(1, np.int64), tabs=np.zeros(0, np.uint32))
    r = ctx.solve(ctx.load(empty), cb.MODE_COUNT)
    assert r.count == 1 and r.nodes == 1 and r.verdict == "SAT"
    q = cspgen.queens(6)
    init = q.full_init()
    init[2, 0] = 0
    r = ctx.solve(ctx.load(q.with_init(init)), cb.MODE_COUNT)
    assert r.count == 0 and r.nodes == 1 and r.fails == 1 and r.verdict == "UNSAT"
    # single variable, no constraints
    one = cspgen.Instance(lo=np.array([3], np.int32), dsize=np.array([5], np.int32),
                          type=np.zeros(0, np.int32), arity=np.zeros(0, np.int32),
                          var_off=np.zeros(1, np.int64), vars=np.zeros(0, np.int32),
                          par_off=np.zeros(1, np.int64), params=np.zeros(0, np.int64),
                          tab_off=np.zeros(1, np.int64), tabs=np.zeros(0, np.uint32))
    r = ctx.solve(ctx.load(one), cb.MODE_ALL, sol_capacity=10)
    assert r.count == 5 and r.nodes == 6 and _canon(r.solutions) == [(v,) for v in range(3, 8)]


def test_limits_and_cap(ctx, cb):
    inst = cspgen.queens(9)
    p = ctx.load(inst)
    r = ctx.solve(p, cb.MODE_COUNT, max_solutions=50)
    assert r.verdict == "LIMIT" and r.count == 50
    r = ctx.solve(p, cb.MODE_ALL, sol_capacity=10)
    assert r.count == 352 and r.n_written == 10 and r.truncated
    for row in r.solutions:
        assert oracle.verify(inst, row)
    r = ctx.solve(p, cb.MODE_COUNT, max_nodes=200, workers=1)
    assert r.verdict == "LIMIT"


def test_split_invariance(ctx, cb):
    inst = cspgen.rb(5, n=16, d=8, dens_pm=300, tight_pm=400)
    p = ctx.load(inst)
    tot = ctx.solve(p, cb.MODE_COUNT)
    parts = 0
    for v in range(8):
        parts += ctx.solve(ctx.load(inst.fix({0: v})), cb.MODE_COUNT).count
    assert parts == tot.count
    assert tot.count == oracle.solve(inst, oracle.MODE_COUNT).count


def test_errors(ctx, cb):
    bad = cspgen.queens(4)
    bad.vars = bad.vars.copy()
    bad.vars[1] = 0  # repeated scope variable
    with pytest.raises(cb.CubicsError):
        ctx.load(bad)


def test_graph_replay_matches_eager(ctx, cb):
    """The captured launch sequence, replayed with eager solves in between,
    gives the eager result every time."""
    inst = cspgen.queens(9)
    ref = oracle.solve(inst, oracle.MODE_COUNT)
    p = ctx.load(inst)
    other = ctx.load(cspgen.queens(7))
    for rep in range(4):
        g = ctx.solve(p, cb.MODE_COUNT, use_graph=True)
        assert (g.count, g.nodes, g.fails) == (ref.count, ref.nodes, ref.fails), rep
        e = ctx.solve(other, cb.MODE_COUNT)
        assert e.count == 40


def test_autotune_then_auto_layout(ctx, cb):
    inst = cspgen.rb(0).fix({0: 3, 1: 5, 2: 7})
    p = ctx.load(inst)
    chosen, div, rates = ctx.autotune([p], cb.MODE_COUNT, time_ms=30, rates=True)
    # n = 40 <= 64, one word per domain: every layout admitted
    assert {lay for lay, _ in rates} == {1, 2, 3}
    # the fastest pair, or one of the same layout with more workers within 5%
    assert rates[(chosen, div)] * 1.05 >= max(rates.values())
    ref = oracle.solve(inst, oracle.MODE_COUNT)
    r = ctx.solve(p, cb.MODE_COUNT)
    assert (r.count, r.nodes) == (ref.count, ref.nodes)


def test_host_cancel_stops_a_running_solve(ctx, cb):
    """cubics_cancel from another thread: the persistent kernel sees the
    pinned flag at its next poll and the solve returns CANCELLED early."""
    import threading
    import time
    p = ctx.load(cspgen.rb(0).fix({0: 0}))  # ~4e10 nodes: tens of seconds uncancelled
    timer = threading.Timer(0.5, ctx.cancel)
    timer.start()
    t0 = time.perf_counter()
    r = ctx.solve(p, cb.MODE_COUNT)
    dt = time.perf_counter() - t0
    timer.join()
    _say(f"cancelled after {dt:.2f} s, {r.nodes} nodes")
    assert r.verdict == "CANCELLED" and dt < 5.0
    # the next solve on the context starts with the flag cleared
    q = ctx.solve(ctx.load(cspgen.queens(8)), cb.MODE_COUNT)
    assert q.verdict == "SAT" and q.count == 92


@pytest.mark.parametrize("layout", LAYOUTS)
def test_two_way_branching(ctx, cb, layout):
    """2-way branching (x = min D_x, then x != min D_x) against the oracle's:
    counts, nodes, fails and solution sets, with donation, a split and one
    worker."""
    inst = cspgen.worked_example(0)
    r = ctx.solve(ctx.load(inst), cb.MODE_ALL, layout=layout, sol_capacity=16, two_way=True)
    assert (r.count, r.nodes, r.fails) == (11, 21, 0)
    for idx in range(30):
        inst = cspgen.mixed(idx + 7100, n=6, dmax=7, m=8)
        _say("two-way mixed", idx, layout)
        ref = oracle.solve(inst, oracle.MODE_ALL, sol_cap=20000, two_way=True)
        r = ctx.solve(ctx.load(inst), cb.MODE_ALL, layout=layout, sol_capacity=max(ref.count, 1),
                      two_way=True)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), idx
        assert _canon(r.solutions) == _canon(ref.solutions), idx
    for idx in range(2):
        inst = cspgen.rb(idx, n=20, d=8, dens_pm=300, tight_pm=390)
        ref = oracle.solve(inst, oracle.MODE_COUNT, two_way=True)
        p = ctx.load(inst)
        # 64 workers donate large subtrees; 2-way paths run deeper than n + 1
        # frames (a variable is branched on again after x != a)
        for kw in ({}, {"split_target": 64}, {"workers": 1}, {"workers": 64}):
            r = ctx.solve(p, cb.MODE_COUNT, layout=layout, two_way=True, **kw)
            assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), (idx, kw)
    q = cspgen.queens(8)
    ref = oracle.solve(q, oracle.MODE_COUNT, two_way=True)
    r = ctx.solve(ctx.load(q), cb.MODE_COUNT, layout=layout, two_way=True, split_target=16)
    assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails)
