"""GPU parity of the all-different propagated to generalized arc consistency
(constraint type 7: maximum matching + strongly connected components on the
device) against the oracle's definition-level version."""
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


def _single(k, lo, d, init):
    inst = cspgen.Instance(
        lo=np.array(lo, np.int32), dsize=np.array([d] * k, np.int32),
        type=np.array([cspgen.ALLDIFF_GAC], np.int32), arity=np.array([k], np.int32),
        var_off=np.array([0, k], np.int64), vars=np.arange(k, dtype=np.int32),
        par_off=np.zeros(2, np.int64), params=np.zeros(0, np.int64),
        tab_off=np.zeros(2, np.int64), tabs=np.zeros(0, np.uint32))
    return inst.with_init(init)


@pytest.mark.parametrize("layout", [1, 2])
def test_gac_root_fixpoints(ctx, cb, layout):
    rng = np.random.default_rng(11)
    for trial in range(80):
        k = int(rng.integers(2, 12))
        d = int(rng.integers(max(2, k - 2), 40))
        lo = [int(v) for v in rng.integers(-3, 4, k)]
        W = (d + 31) // 32
        init = np.zeros((k, W), np.uint32)
        for i in range(k):
            for a in rng.choice(d, size=int(rng.integers(1, min(d, 6) + 1)), replace=False):
                init[i, a // 32] |= np.uint32(1 << (a % 32))
        inst = _single(k, lo, d, init)
        _say("gac root", trial, k, d, layout)
        failed, bits = ctx.root(ctx.load(inst), layout)
        rf, rbits, _ = oracle.root(inst)
        assert failed == rf, trial
        if not rf:
            assert np.array_equal(bits, rbits), trial


@pytest.mark.parametrize("layout", [1, 2])
def test_gac_mixed_counts_nodes(ctx, cb, layout):
    for idx in range(40):
        inst = cspgen.mixed(idx + 4400, n=6, dmax=6, m=7,
                            type_mask=(1 << 5) | (1 << 1) | (1 << 2) | (1 << 3) | (1 << 6)).with_gac()
        _say("gac mixed", idx, layout)
        ref = oracle.solve(inst, oracle.MODE_ALL, sol_cap=5000)
        r = ctx.solve(ctx.load(inst), cb.MODE_ALL, layout=layout, sol_capacity=max(ref.count, 1))
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), idx
        if ref.count <= 5000:
            got = sorted(tuple(int(v) for v in row) for row in r.solutions)
            assert got == sorted(tuple(int(v) for v in row) for row in ref.solutions), idx


def test_gac_global_twins(ctx, cb):
    for idx in range(3):
        inst = cspgen.global_twin(idx).with_gac()
        _say("gac twin", idx)
        ref = oracle.solve(inst, oracle.MODE_COUNT)
        r = ctx.solve(ctx.load(inst), cb.MODE_COUNT)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), idx


def test_gac_is_stronger_on_permutation_puzzles(ctx, cb):
    """k variables over k values with two values forbidden per variable: the
    matching-based all-different prunes at nodes where singleton
    elimination cannot, so the tree shrinks; counts stay equal."""
    rng = np.random.default_rng(5)
    k = 9
    init = np.zeros((k, 1), np.uint32)
    for i in range(k):
        allowed = set(range(k)) - set(rng.choice(k, 2, replace=False).tolist())
        init[i, 0] = sum(1 << a for a in allowed)
    weak = cspgen.Instance(
        lo=np.zeros(k, np.int32), dsize=np.full(k, k, np.int32),
        type=np.array([cspgen.ALLDIFF], np.int32), arity=np.array([k], np.int32),
        var_off=np.array([0, k], np.int64), vars=np.arange(k, dtype=np.int32),
        par_off=np.zeros(2, np.int64), params=np.zeros(0, np.int64),
        tab_off=np.zeros(2, np.int64), tabs=np.zeros(0, np.uint32)).with_init(init)
    gac = weak.with_gac()
    a = ctx.solve(ctx.load(weak), cb.MODE_COUNT)
    b = ctx.solve(ctx.load(gac), cb.MODE_COUNT)
    ra, rb = oracle.solve(weak, oracle.MODE_COUNT), oracle.solve(gac, oracle.MODE_COUNT)
    assert (a.count, a.nodes, a.fails) == (ra.count, ra.nodes, ra.fails)
    assert (b.count, b.nodes, b.fails) == (rb.count, rb.nodes, rb.fails)
    assert a.count == b.count and b.nodes < a.nodes and b.fails == 0


def test_gac_scope_limit(ctx, cb):
    k = 65
    inst = cspgen.Instance(
        lo=np.zeros(k, np.int32), dsize=np.full(k, 70, np.int32),
        type=np.array([cspgen.ALLDIFF_GAC], np.int32), arity=np.array([k], np.int32),
        var_off=np.array([0, k], np.int64), vars=np.arange(k, dtype=np.int32),
        par_off=np.zeros(2, np.int64), params=np.zeros(0, np.int64),
        tab_off=np.zeros(2, np.int64), tabs=np.zeros(0, np.uint32))
    with pytest.raises(Exception) as e:
        ctx.load(inst)
    assert "64" in str(e.value)
